"""Mismatch maximised over a time shift and a phase offset (gw_mismatch_max)
against the oracle's maximisation (a fine inverse-DFT grid refined by a
bounded scalar search), on seeded pairs: plain IMR-form waveforms against a
slightly different system delayed by an off-grid time and rotated by a phase;
broadband random pairs (a sharp overlap peak, no frequency cut); an
identical pair, a pure phase offset and an empty signal.  Window lengths of
2048, 4096, 16384 and 32768 samples (transforms of 1024 to 16384 points)."""

import sys

import numpy as np
import pytest

import oracle
from oracle import surrogate as OS
from oracle import waveform as OW
from paper_2407_19048_amd import gwgen, inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda"
# the kernel forms a_k conj(b_k) / S_k in binary32 and evaluates the phases
# in binary32 after a binary64 range reduction; the oracle works in binary64
TOL = 1e-7

SHAPES = {
    "2048": ("pr1_short", {}),
    "4096": ("pr1_plain", {}),
    "16384": ("paper_scale", {}),
    "32768": ("paper_scale", dict(t_window=16.0)),
}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup(shape):
    name, over = SHAPES[shape]
    cfg = inputs.config(name, **over)
    gen = gwgen.Generator(cfg)
    T = cfg["t_window"]
    F = gen.sizes["F"]
    f = np.arange(F) / T
    S = inputs.true_psd(f, cfg["fs"]).astype(np.float32)
    return cfg, gen, f, S


def _kept(cfg, f, P, i):
    if P is None:
        cut = np.inf
    else:
        _, _, Ms = OW.mass_terms(P[0, i], P[1, i])
        cut = 0.2 / Ms
    k = np.arange(f.size)
    return (f >= cfg["f_min"]) & (k > 0) & (k < f.size - 1) & (f < cut)


def _run(gen, a, b, S, P):
    B = a.shape[0]
    mm = torch.empty(B, dtype=torch.float64, device=DEV)
    mx = torch.empty(B, dtype=torch.float64, device=DEV)
    ta, tb = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    ts = torch.from_numpy(S).to(DEV)
    tp = None if P is None else torch.from_numpy(P).to(DEV)
    gen.mismatch(ta, tb, ts, tp, mm)
    gen.mismatch_max(ta, tb, ts, tp, mx)
    torch.cuda.synchronize()
    return mm.cpu().numpy(), mx.cpu().numpy()


def _check(cfg, f, S, a, b, P, strict, mx, label):
    worst = 0.0
    df = 1.0 / cfg["t_window"]
    for i in range(a.shape[0]):
        kept = _kept(cfg, f, P, i)
        ref = OS.mismatch_maximised(a[i].astype(np.complex128), b[i].astype(np.complex128), S.astype(np.float64),
                                    df, kept)
        d = abs(mx[i] - ref)
        worst = max(worst, d)
        assert d <= TOL, (label, i, mx[i], ref)
        assert mx[i] <= strict[i] + 1e-9, (label, i, mx[i], strict[i])
    _say("%s: B=%d worst |gpu - oracle| %.2e; maximised %s; strict %s"
         % (label, a.shape[0], worst, np.array2string(mx, precision=3), np.array2string(strict, precision=3)))


@pytest.mark.parametrize("shape", sorted(SHAPES))
def test_waveform_pairs_with_time_and_phase_offsets(shape):
    cfg, gen, f, S = _setup(shape)
    B = 5
    _say("waveform pairs, N=%s, B=%d" % (shape, B))
    P, _ = oracle.sample_params(cfg, 31, 0, B, gen.sizes["P"] + gen.sizes["N"])
    rng = np.random.Generator(np.random.PCG64(int(shape)))
    a = np.zeros((B, f.size), np.complex64)
    b = np.zeros_like(a)
    for i in range(B):
        mc, q, c1, c2 = P[0, i], P[1, i], P[2, i], P[3, i]
        ha, _ = OW.fd_waveform(f, 1, mc, q, c1, c2, 1000.0, 0.4, 0.0, cfg["f_min"])
        # a nearby system, delayed by an off-grid time and rotated
        hb, _ = OW.fd_waveform(f, 1, mc * (1.0 + rng.uniform(-2e-4, 2e-4)), q, c1 + rng.uniform(-0.01, 0.01),
                               c2, 1000.0, 0.4, 0.0, cfg["f_min"])
        t0 = rng.choice([-1.0, 1.0]) * rng.uniform(0.01, 0.05)
        ph = rng.uniform(0.5, 2.0 * np.pi - 0.5)
        a[i] = ha
        b[i] = hb * np.exp(1j * ph - 2j * np.pi * f * t0)
    strict, mx = _run(gen, a, b, S, P)
    _check(cfg, f, S, a, b, P, strict, mx, "waveforms N=%s" % shape)
    # the offsets cost most of the strict overlap; maximising recovers it
    assert np.all(strict > 0.1) and np.all(mx < 1e-2)


def test_broadband_pairs_without_cut():
    cfg, gen, f, S = _setup("16384")
    B = 4
    _say("broadband random pairs, no cut, B=%d" % B)
    rng = np.random.Generator(np.random.PCG64(5))
    F = f.size
    a = (rng.standard_normal((B, F)) + 1j * rng.standard_normal((B, F))) * np.sqrt(S)
    t0 = rng.uniform(-0.5, 0.5, (B, 1))
    ph = rng.uniform(0.0, 2.0 * np.pi, (B, 1))
    noise = 0.05 * (rng.standard_normal((B, F)) + 1j * rng.standard_normal((B, F))) * np.sqrt(S)
    b = a * np.exp(1j * ph - 2j * np.pi * f[None, :] * t0) + noise
    a, b = a.astype(np.complex64), b.astype(np.complex64)
    strict, mx = _run(gen, a, b, S, None)
    _check(cfg, f, S, a, b, None, strict, mx, "broadband")


def test_degenerate_pairs():
    cfg, gen, f, S = _setup("16384")
    P, _ = oracle.sample_params(cfg, 32, 0, 3, gen.sizes["P"] + gen.sizes["N"])
    F = f.size
    a = np.zeros((3, F), np.complex64)
    for i in range(3):
        a[i] = OW.fd_waveform(f, 1, P[0, i], P[1, i], P[2, i], P[3, i], 1000.0, 0.4, 0.0, cfg["f_min"])[0]
    b = a.copy()
    b[1] = (a[1] * np.exp(1j * 2.0)).astype(np.complex64)  # pure phase offset
    b[2] = 0.0                                            # empty signal: defined as 0
    _say("degenerate pairs: identical, phase offset, empty")
    strict, mx = _run(gen, a, b, S, P)
    _check(cfg, f, S, a, b, P, strict, mx, "degenerate")
    assert abs(mx[0]) <= 1e-7 and abs(mx[1]) <= 1e-7
    assert strict[1] == pytest.approx(1.0 - np.cos(2.0), abs=1e-6)
    assert mx[2] == 0.0 and strict[2] == 0.0


def test_binary64_transforms_are_rejected():
    cfg = inputs.config("paper_scale", precision=2)
    gen = gwgen.Generator(cfg)
    F = gen.sizes["F"]
    h = torch.zeros((1, F), dtype=torch.complex64, device=DEV)
    S = torch.ones(F, dtype=torch.float32, device=DEV)
    mm = torch.empty(1, dtype=torch.float64, device=DEV)
    with pytest.raises(gwgen.GWError):
        gen.mismatch_max(h, h, S, None, mm)
