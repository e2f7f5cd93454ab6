"""Host-side dense linear algebra of the surrogate's fits (the symmetric
eigen-decomposition behind the reduced basis and the Cholesky solves behind
the skip path and the mismatch head), built on its own with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and checked against numpy:
eigenvalues, eigen-equation residuals and orthonormality on random,
degenerate, diagonal and graded (basis-like) matrices, including n = 1, 2."""

import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "host", "linalg_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("linalg") / "linalg_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-Wall", "-Wextra", "-Werror", "-o", exe, DRIVER]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, tmp_path, mode, payload, nout):
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as fh:
        fh.write(payload)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, mode, fin, fout], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr
    with open(fout, "rb") as fh:
        data = fh.read()
    assert len(data) == nout
    return data


def eig(exe, tmp_path, A):
    n = A.shape[0]
    data = _run(exe, tmp_path, "eig", struct.pack("<i", n) + np.ascontiguousarray(A, "<f8").tobytes(),
                8 * (n + n * n))
    w = np.frombuffer(data[:8 * n], "<f8")
    V = np.frombuffer(data[8 * n:], "<f8").reshape(n, n)
    return w, V


def _check_eig(A, w, V, tol):
    n = A.shape[0]
    scale = max(np.abs(np.linalg.eigvalsh(A)).max(), 1e-300)
    np.testing.assert_allclose(np.sort(w), np.linalg.eigvalsh(A), rtol=0, atol=tol * scale)
    np.testing.assert_allclose(V @ V.T, np.eye(n), rtol=0, atol=tol * n)
    resid = A @ V.T - V.T * w[None, :]
    assert np.abs(resid).max() <= tol * scale * n


def _sym(rs, n):
    X = rs.standard_normal((n, n))
    return 0.5 * (X + X.T)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64])
def test_eig_random_symmetric(driver, tmp_path, n):
    rs = np.random.default_rng(n)
    A = _sym(rs, n)
    w, V = eig(driver, tmp_path, A)
    _check_eig(A, w, V, 1e-12)


def test_eig_degenerate_and_diagonal(driver, tmp_path):
    rs = np.random.default_rng(3)
    u = rs.standard_normal(40)
    A = 2.0 * np.eye(40) + np.outer(u, u)       # 39-fold eigenvalue 2
    w, V = eig(driver, tmp_path, A)
    _check_eig(A, w, V, 1e-12)
    D = np.diag(np.arange(25, dtype=float)[::-1] - 7.0)
    w, V = eig(driver, tmp_path, D)
    _check_eig(D, w, V, 1e-14)
    Z = np.zeros((5, 5))
    w, V = eig(driver, tmp_path, Z)
    assert np.all(w == 0.0)
    np.testing.assert_allclose(V @ V.T, np.eye(5), atol=1e-15)


def test_eig_graded_gram_matrix(driver, tmp_path):
    """Gram matrix of smooth, strongly correlated rows (eigenvalues falling
    over 14 decades, as for the reduced-basis targets): the leading
    eigenpairs are accurate relative to the largest eigenvalue."""
    rs = np.random.default_rng(4)
    x = np.linspace(0, 1, 256)
    rows = np.stack([np.sin(2 * np.pi * (a * x + b)) * np.exp(-c * x)
                     for a, b, c in rs.uniform([0.5, 0, 0], [3, 1, 2], (2000, 3))])
    G = (rows - rows.mean(0)).T @ (rows - rows.mean(0))
    w, V = eig(driver, tmp_path, G)
    _check_eig(G, w, V, 1e-12)
    order = np.argsort(w)[::-1]
    ev, evec = np.linalg.eigh(G)
    for k in range(6):
        v_ref = evec[:, -1 - k]
        assert abs(abs(V[order[k]] @ v_ref) - 1.0) < 1e-9


def test_cholesky_solve(driver, tmp_path):
    rs = np.random.default_rng(5)
    for n, ncol in ((1, 1), (9, 128), (257, 1)):
        X = rs.standard_normal((n + 20, n))
        P = X.T @ X + 1e-3 * np.eye(n)
        R = rs.standard_normal((n, ncol))
        payload = (struct.pack("<ii", n, ncol) + np.ascontiguousarray(P, "<f8").tobytes()
                   + np.ascontiguousarray(R, "<f8").tobytes())
        data = _run(driver, tmp_path, "chol", payload, 4 + 8 * n * ncol)
        assert struct.unpack("<i", data[:4])[0] == 1
        sol = np.frombuffer(data[4:], "<f8").reshape(n, ncol)
        np.testing.assert_allclose(sol, np.linalg.solve(P, R), rtol=1e-9, atol=1e-9 * np.abs(R).max())
    # an indefinite matrix is refused
    payload = struct.pack("<ii", 2, 1) + np.array([[1.0, 2.0], [2.0, 1.0]]).tobytes() + np.ones(2).tobytes()
    data = _run(driver, tmp_path, "chol", payload, 4 + 16)
    assert struct.unpack("<i", data[:4])[0] == 0
