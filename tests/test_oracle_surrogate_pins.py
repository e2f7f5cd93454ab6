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
