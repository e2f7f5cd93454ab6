"""Pins of the surrogate part of the oracle (rounding, backward pass,
mismatch, skip-path linearity)."""

import math

import numpy as np
import pytest

from oracle import surrogate as S
from oracle import waveform


def test_bf16_rounding_matches_library_conversion():
    torch = pytest.importorskip("torch")
    rs = np.random.default_rng(0)
    x = np.concatenate([rs.standard_normal(5000) * 10 ** rs.uniform(-5, 5, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x), ref)


def _rand_weights(rs, scale=0.5):
    dims = [(4, 8), (8, 8), (8, 5)]
    return [(rs.standard_normal(d) * scale, rs.standard_normal(d[1]) * 0.1) for d in dims]


def test_mlp_backward_matches_central_differences():
    rs = np.random.default_rng(1)
    W = _rand_weights(rs)
    x = rs.uniform(-1, 1, (6, 4))
    y = rs.standard_normal((6, 5))

    def loss_of(weights):
        out, _ = S.mlp_forward(weights, x, emulate_bf16=False)
        return S.mse_loss_and_grad(out, y)[0]

    out, cache = S.mlp_forward(W, x, emulate_bf16=False)
    _, dout = S.mse_loss_and_grad(out, y)
    grads = S.mlp_backward(W, cache, dout, emulate_bf16=False)
    h = 1e-6
    for l in range(len(W)):
        for which in (0, 1):
            arr = W[l][which]
            g = grads[l][which]
            for idx in [tuple(rs.integers(0, s) for s in arr.shape) for _ in range(5)]:
                old = arr[idx]
                arr[idx] = old + h
                lp = loss_of(W)
                arr[idx] = old - h
                lm = loss_of(W)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - g[idx]) < 1e-7 + 1e-6 * abs(g[idx])


def test_silu_gradient():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    np.testing.assert_allclose(S.silu_grad(z), (S.silu(z + h) - S.silu(z - h)) / (2 * h), atol=1e-8)


def _toy_signal(n=2048):
    f = np.arange(n) * 0.25
    rs = np.random.default_rng(2)
    h = (f + 1.0) ** (-7.0 / 6.0) * np.exp(1j * rs.uniform(0, 2 * np.pi, n))
    S_ = 1.0 + (f / 100.0) ** 2
    kept = (f > 10) & (f < 400)
    return h, S_, kept


def test_mismatch_identities():
    h, S_, kept = _toy_signal()
    assert abs(S.mismatch(h, h, S_, 0.25, kept)) < 1e-15
    assert abs(S.mismatch(3.7 * h, h, S_, 0.25, kept)) < 1e-15
    # a constant phase offset phi gives mm = 1 - cos(phi)
    assert abs(S.mismatch(h * np.exp(0.3j), h, S_, 0.25, kept) - (1 - math.cos(0.3))) < 1e-14


def test_mismatch_small_phase_error_law():
    h, S_, kept = _toy_signal()
    rs = np.random.default_rng(3)
    dphi = 1e-3 * rs.standard_normal(h.shape[0])
    mm = S.mismatch(h * np.exp(1j * dphi), h, S_, 0.25, kept)
    w = np.abs(h[kept]) ** 2 / S_[kept]
    m = np.sum(w * dphi[kept]) / np.sum(w)
    var_w = np.sum(w * (dphi[kept] - m) ** 2) / np.sum(w)
    # to second order mm = (weighted mean of dphi^2)/2 - ..., i.e. Var_w/2 plus
    # the mean term m^2/2 that a constant offset would add
    assert abs(mm - 0.5 * (var_w + m * m)) < 1e-3 * mm


def test_maximised_mismatch_removes_time_shift_and_phase():
    h, S_, kept = _toy_signal()
    df = 0.25
    k = np.arange(h.shape[0])
    assert abs(S.mismatch_maximised(h, h, S_, df, kept)) < 1e-12
    # a phase offset and a time shift off the search grid are both undone
    tau0 = 0.123456789  # in window lengths
    g = 2.5 * h * np.exp(0.7j) * np.exp(-2j * np.pi * k * tau0)
    assert S.mismatch(g, h, S_, df, kept) > 0.5
    assert abs(S.mismatch_maximised(g, h, S_, df, kept)) < 1e-10
    assert abs(S.mismatch_maximised(h, g, S_, df, kept)) < 1e-10


def test_maximised_mismatch_bounds_and_brute_force():
    h, S_, kept = _toy_signal(256)
    df = 0.25
    rs = np.random.default_rng(5)
    g = h * np.exp(1j * 0.05 * rs.standard_normal(h.shape[0]))
    strict = S.mismatch(g, h, S_, df, kept)
    best = S.mismatch_maximised(g, h, S_, df, kept)
    assert 0.0 <= best <= strict
    # brute force: |c| on a direct grid of shifts over the whole window, then
    # on a second direct grid of the same size around the first's best
    kk = np.nonzero(kept)[0]
    z = g[kk] * np.conj(h[kk]) / S_[kk]

    def cmax(taus):
        c = np.abs(np.exp(2j * np.pi * np.outer(taus, kk)) @ z)
        return taus[np.argmax(c)], c.max()

    t0, _ = cmax(np.linspace(0.0, 1.0, 20001))
    _, cm = cmax(np.linspace(t0 - 5e-5, t0 + 5e-5, 20001))
    aa = np.sum(np.abs(g[kk]) ** 2 / S_[kk])
    bb = np.sum(np.abs(h[kk]) ** 2 / S_[kk])
    brute = 1.0 - cm / math.sqrt(aa * bb)
    assert best <= brute + 1e-12  # the search finds at least the grid's best
    assert brute - best < 1e-10   # and no more than the fine grid's


def test_interp_nodes_exact_for_linear_in_log_mf():
    Mf = S.node_grid()
    vals = 3.0 + 2.0 * np.log(Mf)
    Ms = 1e-3
    f = np.geomspace(S.MF_LO / Ms * 1.01, S.MF_HI / Ms * 0.99, 50)
    np.testing.assert_allclose(S.interp_nodes(vals, Ms, f), 3.0 + 2.0 * np.log(Ms * f), rtol=1e-12)


def test_phase_residual_is_linear_in_skip_features_below_merger():
    """Below f_t the residual P - P_N at a fixed Mf node is an exact linear
    function of the skip-path features, with coefficients that depend on
    v = (pi Mf)^(1/3) only."""
    rs = np.random.default_rng(4)
    Mf = S.node_grid()
    j = 40  # Mf ~ 2.4e-3: inspiral for every system in the prior
    v = np.cbrt(math.pi * Mf[j])
    coef = np.array([v ** -3, v ** -2, v ** -1, 1.0, v, v ** 2, math.log(v), v * math.log(v), 0.0])
    for _ in range(30):
        mc, q = rs.uniform(10, 100), rs.uniform(0.125, 1)
        c1, c2 = rs.uniform(-0.99, 0.99, 2)
        ratio, dpsi = S.targets(mc, q, c1, c2)
        phi = S.features(q, c1, c2)
        f_rd, _ = waveform.ringdown_frequencies(mc, q, c1, c2)
        eta, M, Ms = waveform.mass_terms(mc, q)
        assert Mf[j] / Ms < 0.5 * f_rd
        assert ratio[j] == 1.0
        assert abs(dpsi[j] - phi @ coef) < 1e-9 * max(1.0, abs(dpsi[j]))


# ------------------------------------------------------------- optimiser

def test_adamw_first_step_by_hand():
    """At t = 1 with zero moments, m_hat = g and v_hat = g^2, so each weight
    moves by lr (sign(g) + wd p) (|g| >> eps).  Values worked by hand for
    p = (1, -2, 0.5), g = (0.3, -4, 0), lr = 0.01, wd = 0.1."""
    p, m, v = S.adamw_step([1.0, -2.0, 0.5], [0.3, -4.0, 0.0], np.zeros(3), np.zeros(3), 1, 0.01, 0.1)
    np.testing.assert_allclose(p, [0.989, -1.988, 0.4995], rtol=0, atol=1e-9)
    np.testing.assert_allclose(m, [0.03, -0.4, 0.0], rtol=1e-15, atol=0)
    np.testing.assert_allclose(v, [0.00009, 0.016, 0.0], rtol=1e-12, atol=0)


def _adam_kingma_ba(p, grads, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam in the rearranged form of Kingma & Ba (2015), section 2: the bias
    corrections folded into the step size alpha_t = alpha sqrt(1 - beta2^t) /
    (1 - beta1^t), with eps_hat = eps sqrt(1 - beta2^t) so that it is the same
    update as with bias-corrected moments."""
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t, g in enumerate(grads, start=1):
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        a_t = lr * math.sqrt(1 - beta2 ** t) / (1 - beta1 ** t)
        p = p - a_t * m / (np.sqrt(v) + eps * math.sqrt(1 - beta2 ** t))
    return p


def test_adamw_without_decay_is_adam():
    rs = np.random.default_rng(5)
    p0 = rs.standard_normal(50)
    grads = [rs.standard_normal(50) * 10 ** rs.uniform(-3, 1) for _ in range(25)]
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        p, m, v = S.adamw_step(p, g, m, v, t, 3e-3, 0.0)
    np.testing.assert_allclose(p, _adam_kingma_ba(p0, grads, 3e-3), rtol=1e-12, atol=1e-14)


def test_adamw_decay_is_decoupled_from_the_gradient():
    """With zero gradients the moments stay zero and the weights decay
    geometrically by (1 - lr wd) per step; an L2 penalty folded into the
    gradient would instead be normalised by Adam into steps of about lr."""
    p0 = np.array([3.0, -0.25, 1e-3])
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 101):
        p, m, v = S.adamw_step(p, np.zeros(3), m, v, t, 0.01, 0.5)
    np.testing.assert_allclose(p, p0 * (1 - 0.005) ** 100, rtol=1e-12)
    assert np.all(m == 0) and np.all(v == 0)


def test_adam_step_is_invariant_to_gradient_scale():
    rs = np.random.default_rng(6)
    p0 = rs.standard_normal(20)
    grads = [rs.standard_normal(20) for _ in range(5)]
    a, b = p0.copy(), p0.copy()
    ma = va = mb = vb = np.zeros(20)
    for t, g in enumerate(grads, start=1):
        a, ma, va = S.adamw_step(a, g, ma, va, t, 1e-2, 0.01)
        b, mb, vb = S.adamw_step(b, 1000.0 * g, mb, vb, t, 1e-2, 0.01)
    np.testing.assert_allclose(a, b, rtol=1e-7, atol=1e-10)


# ------------------------------------------------------- ridge mismatch head

def test_ridge_head_hand_solved_case():
    """h = (-1, 1), y = (0, 2): X^T X = 2 I and X^T y = (2, 2), so with the
    penalty ridge n = 2 ridge on both coefficients w = (1, 1) / (1 + ridge)."""
    w = S.ridge_head(np.array([[-1.0], [1.0]]), np.array([0.0, 2.0]), 0.5)
    np.testing.assert_allclose(w, [2.0 / 3.0, 2.0 / 3.0], rtol=1e-14)
    w0 = S.ridge_head(np.array([[-1.0], [1.0]]), np.array([0.0, 2.0]), 0.0)
    np.testing.assert_allclose(w0, [1.0, 1.0], rtol=1e-14)


def test_ridge_head_satisfies_its_normal_equations():
    rs = np.random.default_rng(7)
    n, k, lam = 300, 12, 1e-2
    h = rs.standard_normal((n, k))
    y = h @ rs.standard_normal(k) + 0.3 + 0.1 * rs.standard_normal(n)
    w = S.ridge_head(h, y, lam)
    X = np.concatenate([h, np.ones((n, 1))], axis=1)
    grad = X.T @ (X @ w - y) + lam * n * w
    assert np.abs(grad).max() < 1e-9 * np.abs(X.T @ y).max()


# ------------------------------------------------------------ reduced basis

def test_reduced_basis_rank_one_and_sign():
    """Rows that are multiples of one unit vector u (plus a common offset)
    give u itself as the first basis vector, sign fixed by the largest-
    magnitude component (here negative in u, so the vector is -u)."""
    u = np.array([0.1, -0.9, 0.3, 0.2, -0.2])
    u = u / np.linalg.norm(u)
    c = np.array([1.0, -3.0, 0.5, 2.0, 7.0, -1.5])
    X = 4.0 + c[:, None] * u[None, :]
    mean, V = S.reduced_basis(X, 1)
    np.testing.assert_allclose(mean, 4.0 + c.mean() * u, atol=1e-14)
    np.testing.assert_allclose(V[0], -u, atol=1e-12)
    assert S.truncation_error(X, mean, V) < 1e-24


def test_reduced_basis_eckart_young():
    """The truncation error of the leading k vectors equals the sum of the
    discarded squared singular values (from the full spectrum of X - mean
    computed by the eigenvalues of its Gram matrix), no random orthonormal
    basis of the same size does better, and the vectors are orthonormal."""
    rs = np.random.default_rng(8)
    n, dim, k = 400, 60, 8
    scales = 2.0 ** -np.arange(dim / 2, step=0.5)
    X = (rs.standard_normal((n, dim)) * scales) @ np.linalg.qr(rs.standard_normal((dim, dim)))[0]
    mean, V = S.reduced_basis(X, k)
    ev = np.sort(np.linalg.eigvalsh((X - mean).T @ (X - mean)))[::-1]
    err = S.truncation_error(X, mean, V)
    assert abs(err - ev[k:].sum()) < 1e-9 * ev.sum()
    np.testing.assert_allclose(V @ V.T, np.eye(k), atol=1e-12)
    for _ in range(20):
        Q = np.linalg.qr(rs.standard_normal((dim, k)))[0].T
        assert S.truncation_error(X, mean, Q) >= err
    big = V[np.arange(k), np.argmax(np.abs(V), axis=1)]
    assert np.all(big > 0)


def test_routing_sends_nan_to_the_plain_model():
    keep = S.keeps_surrogate(np.array([-5.0, -3.0, -2.9, np.nan, np.inf, -np.inf]), -3.0)
    assert keep.tolist() == [True, True, False, False, False, True]


@pytest.mark.parametrize("iota", [0.3, 1.5707963, 2.6, 3.14159])
def test_reconstruction_polarisations_follow_the_plain_model(iota):
    """With node values equal to the plain model's exact targets, the
    reconstructed plus AND cross polarisations approach the plain model's
    (fd_waveform, a separate code path), at every inclination including edge
    on (cos iota ~ 0) and face off (iota ~ pi)."""
    from oracle import pipeline
    from paper_2407_19048_amd import inputs
    cfg = inputs.config("surrogate")
    p = np.zeros(12)
    p[:5] = (35.0, 0.6, 0.2, -0.4, 500.0)
    p[5], p[9] = iota, 1.1
    r, d = S.targets(p[0], p[1], p[2], p[3])
    hp, hc = S.reconstruct(cfg, p, r, d)
    hp_o, hc_o = pipeline.waveform_on_grid(cfg, p)
    e_p = np.linalg.norm(hp - hp_o) / np.linalg.norm(hp_o)
    assert e_p < 2e-3
    if abs(math.cos(iota)) > 1e-6:
        e_c = np.linalg.norm(hc - hc_o) / np.linalg.norm(hc_o)
        assert e_c < 2e-3 and abs(e_c - e_p) < 1e-9
    else:
        assert np.abs(hc).max() <= 1e-6 * np.abs(hp).max()
