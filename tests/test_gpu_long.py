"""Windows longer than 32768 samples (four-step transforms through HBM)
against the oracle: the fused batch for every split NC = N1 x N2 (rows of
N1 = 8192 with N2 = 4, 8, 16, 32 for N = 2^16 ... 2^19, rows of 16384 with
N2 = 32 for N = 2^20), the benchmark's batch of 256 at N = 2^19 (sampled),
sine-Gaussian bursts, and the inject and whiten steps (whitened relative L2
per window <= 1e-5)."""

import sys

import numpy as np
import pytest

import oracle
from oracle import pipeline
from paper_2407_19048_amd import gwgen, inputs
from draws import checked_draws

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


_BG = {}


def bg_for(fs, log2):
    key = (fs, log2)
    if key not in _BG:
        _BG[key] = inputs.background(3, 1 << log2, fs, seed=1)
    return _BG[key]


@pytest.mark.parametrize("T", [32.0, 64.0, 128.0, 256.0, 512.0])
def test_long_fused_batch_matches_oracle(T):
    cfg = inputs.config("bns_long", t_window=T)
    N = int(T * cfg["fs"])
    bg_np = bg_for(2048.0, 22)
    gen = gwgen.Generator(cfg)
    B = 2
    out = torch.empty((B, 3, N), dtype=torch.float32, device=DEV)
    st = torch.zeros(B, dtype=torch.int32, device=DEV)
    ws = gen.alloc_workspace(B)
    N1 = 8192 if N <= (1 << 19) else 16384
    _say("long fused T=%g N=%d N1=%d N2=%d" % (T, N, N1, N // (2 * N1)))
    gen.generate_batch(5, 1, B, torch.from_numpy(bg_np).to(DEV), out, ws, status=st)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    P, O, G = params.cpu().numpy(), offs.cpu().numpy(), out.cpu().numpy()
    P, O = checked_draws(cfg, 5, 1 * B, P, O, bg_np.shape[1])
    worst = 0.0
    for i in range(B):
        ref = pipeline.generate_sample(cfg, bg_np, P[:, i], int(O[i]))
        for d in range(3):
            e = rel_l2(G[i, d], ref[d])
            worst = max(worst, e)
            assert e <= 1e-5, (T, i, d, e)
    _say("long fused worst rel L2 %.3e" % worst)
    assert (st.cpu().numpy() & ~gwgen.STATUS_CUT_AT_NYQUIST).max() == 0


def test_long_full_size_sampled():
    """Batch 256 of 256 s windows (N = 2^19) after the autotuner, as the
    benchmark launches it; four samples checked against the oracle in full
    and the whole batch for finite output and status bits."""
    cfg = inputs.config("bns_long")
    N = int(cfg["t_window"] * cfg["fs"])
    B = cfg["batch"]
    bg_np = bg_for(2048.0, 22)
    bg = torch.from_numpy(bg_np).to(DEV)
    gen = gwgen.Generator(cfg)
    out = torch.empty((B, 3, N), dtype=torch.float32, device=DEV)
    st = torch.zeros(B, dtype=torch.int32, device=DEV)
    ws = gen.alloc_workspace(B)
    _say("long full size B=%d N=%d" % (B, N))
    gen.autotune(B, bg, out, ws, reps=1)
    gen.generate_batch(2, 0, B, bg, out, ws, status=st)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    P, O = params.cpu().numpy(), offs.cpu().numpy()
    idx = (0, 1, B // 2, B - 1)
    P, O = checked_draws(cfg, 2, 0, P, O, bg_np.shape[1], idx=idx)
    worst = 0.0
    for i in idx:
        ref = pipeline.generate_sample(cfg, bg_np, P[:, i], int(O[i]))
        got = out[i].cpu().numpy()
        for d in range(3):
            e = rel_l2(got[d], ref[d])
            worst = max(worst, e)
            assert e <= 1e-5, (i, d, e)
    _say("long full size worst rel L2 %.3e" % worst)
    assert bool(torch.isfinite(out).all())
    assert (st.cpu().numpy() & ~gwgen.STATUS_CUT_AT_NYQUIST).max() == 0


def test_long_sine_gaussian_matches_oracle():
    """Sine-Gaussian bursts in 64 s windows (N = 2^17, four-step path)."""
    cfg = inputs.config("sine_gaussian", t_window=64.0)
    N = int(cfg["t_window"] * cfg["fs"])
    bg_np = bg_for(2048.0, 22)
    gen = gwgen.Generator(cfg)
    B = 3
    out = torch.empty((B, 3, N), dtype=torch.float32, device=DEV)
    ws = gen.alloc_workspace(B)
    _say("long sine-Gaussian N=%d" % N)
    gen.generate_batch(9, 0, B, torch.from_numpy(bg_np).to(DEV), out, ws)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    P, O, G = params.cpu().numpy(), offs.cpu().numpy(), out.cpu().numpy()
    P, O = checked_draws(cfg, 9, 0, P, O, bg_np.shape[1])
    worst = 0.0
    for i in range(B):
        ref = pipeline.generate_sample(cfg, bg_np, P[:, i], int(O[i]))
        for d in range(3):
            e = rel_l2(G[i, d], ref[d])
            worst = max(worst, e)
            assert e <= 1e-5, (i, d, e)
    _say("long sine-Gaussian worst rel L2 %.3e" % worst)


def test_long_binary32_mode_transforms():
    """Precision mode 0 (binary32 phase) on the four-step path: with the
    sources placed so far away that the signal is below 1e-12 of the noise,
    the whitened windows test the binary32 transforms, Welch sums and gains
    against the oracle at the usual bar; the phase precision is irrelevant."""
    cfg = inputs.config("bns_long", t_window=64.0, precision=0, dl=(1e12, 2e12))
    N = int(cfg["t_window"] * cfg["fs"])
    bg_np = bg_for(2048.0, 22)
    gen = gwgen.Generator(cfg)
    B = 2
    out = torch.empty((B, 3, N), dtype=torch.float32, device=DEV)
    ws = gen.alloc_workspace(B)
    _say("long binary32 mode N=%d" % N)
    gen.generate_batch(4, 0, B, torch.from_numpy(bg_np).to(DEV), out, ws)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    P, O, G = params.cpu().numpy(), offs.cpu().numpy(), out.cpu().numpy()
    P, O = checked_draws(cfg, 4, 0, P, O, bg_np.shape[1])
    worst = 0.0
    for i in range(B):
        ref = pipeline.generate_sample(cfg, bg_np, P[:, i], int(O[i]))
        for d in range(3):
            e = rel_l2(G[i, d], ref[d])
            worst = max(worst, e)
            assert e <= 1e-5, (i, d, e)
    _say("long binary32 mode worst rel L2 %.3e" % worst)


def test_long_inject_and_whiten_steps_match_oracle():
    cfg = inputs.config("bns_long", t_window=128.0)
    bg_np = bg_for(2048.0, 22)
    gen = gwgen.Generator(cfg)
    z = gen.sizes
    B = 2
    bg = torch.from_numpy(bg_np).to(DEV)
    params = torch.empty((12, B), dtype=torch.float64, device=DEV)
    offs = torch.empty(B, dtype=torch.int64, device=DEV)
    gen.sample_params(7, 0, B, bg_np.shape[1], params, offs)
    hp = torch.empty((B, z["F"]), dtype=torch.complex64, device=DEV)
    hc = torch.empty_like(hp)
    gen.gen_fd_waveform(params, hp, hc)
    hdet = torch.empty((B, 3, z["F"]), dtype=torch.complex64, device=DEV)
    gen.project_detectors(params, hp, hc, hdet)
    strain = torch.empty((B, 3, z["N"]), dtype=torch.float32, device=DEV)
    gen.inject(bg, offs, hdet, strain)
    psd = torch.empty((B, 3, z["Fw"]), dtype=torch.float32, device=DEV)
    gen.welch_psd(bg, offs, psd)
    out = torch.empty_like(strain)
    gen.whiten(strain, psd, out)
    torch.cuda.synchronize()
    P, O = checked_draws(cfg, 7, 0, params.cpu().numpy(), offs.cpu().numpy(), bg_np.shape[1])
    S, W = strain.cpu().numpy(), out.cpu().numpy()
    for i in range(B):
        ref, stg = pipeline.generate_sample(cfg, bg_np, P[:, i], int(O[i]), return_stages=True)
        for d in range(3):
            assert rel_l2(S[i, d], stg["y"][d]) <= 1e-6, (i, d)
            assert rel_l2(W[i, d], ref[d]) <= 1e-5, (i, d)


def test_long_windows_reject_unsupported_paths():
    cfg = inputs.config("bns_long", t_window=64.0)
    gen = gwgen.Generator(cfg)
    with pytest.raises(gwgen.GWError):
        gen.whiten_filter(torch.ones((3, gen.sizes["Fw"]), dtype=torch.float32, device=DEV), 64,
                          torch.empty((3, gen.sizes["F"]), dtype=torch.float32, device=DEV))


@pytest.mark.parametrize("structure", [0, 1])
def test_long_window_structures_match_oracle(structure):
    """Both structures of the four-step window stage (0: row transforms, bins
    and inverse rows as three passes; 1: fused per row pair) against the
    oracle, at N2 = 8 (rows 0 and 4 self-paired, rows 1-3 paired with 7-5)."""
    cfg = inputs.config("bns_long", t_window=128.0)
    N = int(cfg["t_window"] * cfg["fs"])
    bg_np = bg_for(2048.0, 22)
    gen = gwgen.Generator(cfg)
    gen.set_tuning(gwgen.TUNE_ORD_WINDOW, structure)
    B = 2
    out = torch.empty((B, 3, N), dtype=torch.float32, device=DEV)
    ws = gen.alloc_workspace(B)
    _say("long structure %d N=%d" % (structure, N))
    gen.generate_batch(6, 2, B, torch.from_numpy(bg_np).to(DEV), out, ws)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    P, O = checked_draws(cfg, 6, 2 * B, params.cpu().numpy(), offs.cpu().numpy(), bg_np.shape[1])
    G = out.cpu().numpy()
    worst = 0.0
    for i in range(B):
        ref = pipeline.generate_sample(cfg, bg_np, P[:, i], int(O[i]))
        for d in range(3):
            e = rel_l2(G[i, d], ref[d])
            worst = max(worst, e)
            assert e <= 1e-5, (structure, i, d, e)
    _say("long structure %d worst rel L2 %.3e" % (structure, worst))
