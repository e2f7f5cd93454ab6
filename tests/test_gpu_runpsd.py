"""Per-run PSD mode through the C ABI against the oracle: the run PSD (RMS
of gpu/oracle - 1 <= 1e-4), the truncated whitening filter from a PSD given
to both sides (relative L2 <= 1e-5), and batches whitened with that filter
(relative L2 per window <= 1e-5, params and offsets equal to the plain
batch's draws)."""

import math
import sys

import numpy as np
import pytest

from oracle import pipeline
from paper_2407_19048_amd import gwgen, inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


_BG = {}


def bg_for(name, log2):
    key = (name, log2)
    if key not in _BG:
        cfg = inputs.config(name)
        _BG[key] = inputs.background(len(cfg["det_ids"]), 1 << log2, cfg["fs"], seed=1)
    return _BG[key]


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("name,n_chunks", [("pr1_plain", 3), ("paper_scale", 5)])
def test_run_psd_matches_oracle(name, n_chunks):
    cfg = inputs.config(name)
    bg_np = bg_for(name, 21)
    gen = gwgen.Generator(cfg)
    psd = torch.empty((gen.sizes["D"], gen.sizes["Fw"]), dtype=torch.float32, device=DEV)
    _say("run psd %s n_chunks=%d" % (name, n_chunks))
    ws = gen.run_psd(_gpu(bg_np), n_chunks, psd)
    torch.cuda.synchronize()
    del ws
    ref = pipeline.run_psds(cfg, bg_np, n_chunks)
    got = psd.cpu().numpy().astype(np.float64)
    for d in range(ref.shape[0]):
        rms = math.sqrt(np.mean((got[d] / ref[d] - 1.0) ** 2))
        assert rms <= 1e-4, (d, rms)


def _oracle_filter_inputs(cfg, n_chunks, M, log2=21):
    bg_np = bg_for("paper_scale" if cfg["fs"] == 2048.0 else "pr1_plain", log2)
    psd = pipeline.run_psds(cfg, bg_np, n_chunks).astype(np.float32)
    filt = pipeline.run_filters(cfg, psd.astype(np.float64), M)
    return bg_np, psd, filt


@pytest.mark.parametrize("name,M", [("pr1_plain", 1024), ("pr1_short", 512), ("paper_scale", 4096),
                                    ("paper_scale", 2)])
def test_whiten_filter_matches_oracle(name, M):
    cfg = inputs.config(name)
    _, psd, ref = _oracle_filter_inputs(cfg, 3, M)
    gen = gwgen.Generator(cfg)
    filt = torch.empty((gen.sizes["D"], gen.sizes["F"]), dtype=torch.float32, device=DEV)
    _say("whiten filter %s M=%d" % (name, M))
    gen.whiten_filter(_gpu(psd), M, filt)
    torch.cuda.synchronize()
    got = filt.cpu().numpy()
    for d in range(ref.shape[0]):
        assert rel_l2(got[d], ref[d]) <= 1e-5, (d, rel_l2(got[d], ref[d]))


def test_whiten_filter_status_bits():
    """A NaN PSD bin in one detector and a zero bin in another are dropped
    from the gain and reported per detector; the clean detector reports 0."""
    cfg = inputs.config("paper_scale")
    _, psd, _ = _oracle_filter_inputs(cfg, 3, 4096)
    bad = psd.copy()
    bad[0, 300] = np.nan   # 300 * df = 150 Hz, inside the kept band
    bad[1, 500] = 0.0
    gen = gwgen.Generator(cfg)
    filt = torch.empty((gen.sizes["D"], gen.sizes["F"]), dtype=torch.float32, device=DEV)
    status = torch.full((gen.sizes["D"],), -1, dtype=torch.int32, device=DEV)  # overwritten
    gen.whiten_filter(_gpu(bad), 4096, filt, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy().astype(np.uint32)
    _say("whiten filter status bits %s" % st.tolist())
    assert st.tolist() == [gwgen.STATUS_NONFINITE_PSD, gwgen.STATUS_NONPOSITIVE_PSD, 0]
    assert bool(torch.isfinite(filt).all())


def _run_batch(gen, bg, filt, crop, B, seed=9, batch_index=1):
    N = gen.sizes["N"]
    out = torch.empty((B, gen.sizes["D"], N - 2 * crop), dtype=torch.float32, device=DEV)
    ws = gen.alloc_workspace(B)
    gen.generate_batch_runpsd(seed, batch_index, B, bg, filt, crop, out, ws)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    return out.cpu().numpy(), params.cpu().numpy(), offs.cpu().numpy()


@pytest.mark.parametrize("name,M,crop", [("paper_scale", 4096, 2048), ("pr1_plain", 1024, 512),
                                         ("pr1_short", 512, 256), ("paper_scale", 4096, 0),
                                         ("paper_scale", 64, 8188)])
def test_runpsd_batch_matches_oracle(name, M, crop):
    cfg = inputs.config(name)
    bg_np, _, filt = _oracle_filter_inputs(cfg, 3, M)
    gen = gwgen.Generator(cfg)
    B = 8
    _say("runpsd batch %s M=%d crop=%d" % (name, M, crop))
    bg = _gpu(bg_np)
    out, params, offs = _run_batch(gen, bg, _gpu(filt.astype(np.float32)), crop, B)
    # the draws are those of the plain batch with the same seed and index
    ref_p, ref_o = pipeline.sample_params(cfg, 9, 1 * B, B, bg_np.shape[1])
    np.testing.assert_allclose(params, ref_p, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(offs, ref_o)
    f32 = filt.astype(np.float32).astype(np.float64)
    worst = 0.0
    for i in range(B):
        ref = pipeline.generate_sample_runpsd(cfg, bg_np, ref_p[:, i], int(ref_o[i]), f32, crop)
        for d in range(ref.shape[0]):
            e = rel_l2(out[i, d], ref[d])
            worst = max(worst, e)
            assert e <= 1e-5, (i, d, e)
    _say("runpsd worst rel L2 %.3e" % worst)


def test_runpsd_full_size_sampled():
    cfg = inputs.config("paper_scale")
    M, crop = 4096, 2048
    bg_np, _, filt = _oracle_filter_inputs(cfg, 3, M, log2=22)
    gen = gwgen.Generator(cfg)
    B = 2048
    out, params, offs = _run_batch(gen, _gpu(bg_np), _gpu(filt.astype(np.float32)), crop, B, seed=2, batch_index=0)
    # the GPU draws are the oracle's before they are handed to it
    idx = np.array([0, 777, B - 1])
    ref_p, ref_o = pipeline.sample_params(cfg, 2, 0, B, bg_np.shape[1])
    np.testing.assert_allclose(params[:, idx], ref_p[:, idx], rtol=1e-12, atol=0)
    np.testing.assert_array_equal(offs, ref_o)
    f32 = filt.astype(np.float32).astype(np.float64)
    for i in idx:
        ref = pipeline.generate_sample_runpsd(cfg, bg_np, params[:, i], int(offs[i]), f32, crop)
        for d in range(3):
            assert rel_l2(out[i, d], ref[d]) <= 1e-5
    # whitened noise-dominated windows: unit variance over the kept band
    v = float(np.var(out))
    _say("runpsd full size: output variance %.4f" % v)
    assert 0.8 < v < 1.2


def test_runpsd_rejects_bad_arguments():
    cfg = inputs.config("pr1_plain")
    gen = gwgen.Generator(cfg)
    psd = torch.ones((gen.sizes["D"], gen.sizes["Fw"]), dtype=torch.float32, device=DEV)
    filt = torch.empty((gen.sizes["D"], gen.sizes["F"]), dtype=torch.float32, device=DEV)
    for M in (0, 3, gen.sizes["N"]):
        with pytest.raises(gwgen.GWError):
            gen.whiten_filter(psd, M, filt)
    bg = torch.zeros((gen.sizes["D"], 1 << 16), dtype=torch.float32, device=DEV)
    with pytest.raises(gwgen.GWError):
        gen.run_psd(bg, 1000, psd)  # stretches beyond the background
