"""View pairs and extrinsic oversampling through the C ABI against the
oracle (whitened relative L2 per window <= 1e-5, params relative error <=
1e-12, offsets exact)."""

import sys

import numpy as np
import pytest

from oracle import pipeline, priors
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


@pytest.mark.parametrize("name", ["pr1_plain", "pr1_short", "paper_scale"])
def test_view_pairs_match_oracle(name):
    cfg = inputs.config(name)
    bg_np = bg_for(name, 21)
    gen = gwgen.Generator(cfg)
    B, D, N = 8, gen.sizes["D"], gen.sizes["N"]
    bg = torch.from_numpy(bg_np).to(DEV)
    ref_t = torch.empty((B, D, N), dtype=torch.float32, device=DEV)
    shf_t = torch.empty_like(ref_t)
    ws = gen.alloc_workspace(B)
    _say("view pairs %s" % name)
    gen.generate_batch_pairs(6, 2, B, bg, ref_t, shf_t, ws)
    plain = torch.empty_like(ref_t)
    ws2 = gen.alloc_workspace(B)
    gen.generate_batch(6, 2, B, bg, plain, ws2)
    torch.cuda.synchronize()
    # the shifted view is the ordinary batch, bit for bit
    assert torch.equal(shf_t, plain)
    p, o = priors.sample_params(cfg, 6, 2 * B, B, bg_np.shape[1])
    got_ref, got_shf = ref_t.cpu().numpy(), shf_t.cpu().numpy()
    worst = 0.0
    for i in range(B):
        d_ref, d_shf = pipeline.generate_pair(cfg, bg_np, p[:, i], int(o[i]))
        for d in range(D):
            e = max(rel_l2(got_ref[i, d], d_ref[d]), rel_l2(got_shf[i, d], d_shf[d]))
            worst = max(worst, e)
            assert e <= 1e-5, (i, d, e)
    _say("view pairs worst rel L2 %.3e" % worst)


def test_view_pairs_full_size_sampled():
    """The benchmark's batch of 2048 pairs at the paper-scale shape; four
    pairs checked against the oracle, the whole batch for finite output."""
    cfg = inputs.config("paper_scale")
    bg_np = bg_for("paper_scale", 22)
    gen = gwgen.Generator(cfg)
    B, D, N = cfg["batch"], gen.sizes["D"], gen.sizes["N"]
    bg = torch.from_numpy(bg_np).to(DEV)
    ref_t = torch.empty((B, D, N), dtype=torch.float32, device=DEV)
    shf_t = torch.empty_like(ref_t)
    ws = gen.alloc_workspace(B)
    _say("view pairs full size B=%d" % B)
    gen.generate_batch_pairs(3, 0, B, bg, ref_t, shf_t, ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(ref_t).all()) and bool(torch.isfinite(shf_t).all())
    p, o = priors.sample_params(cfg, 3, 0, B, bg_np.shape[1])
    worst = 0.0
    for i in (0, 1, B // 2, B - 1):
        d_ref, d_shf = pipeline.generate_pair(cfg, bg_np, p[:, i], int(o[i]))
        g_ref, g_shf = ref_t[i].cpu().numpy(), shf_t[i].cpu().numpy()
        for d in range(D):
            e = max(rel_l2(g_ref[d], d_ref[d]), rel_l2(g_shf[d], d_shf[d]))
            worst = max(worst, e)
            assert e <= 1e-5, (i, d, e)
    _say("view pairs full size worst rel L2 %.3e" % worst)


@pytest.mark.parametrize("ext_k", [1, 4])
def test_oversampled_batch_matches_oracle(ext_k):
    cfg = inputs.config("paper_scale")
    bg_np = bg_for("paper_scale", 21)
    gen = gwgen.Generator(cfg)
    B, D, N = 12, gen.sizes["D"], gen.sizes["N"]
    bg = torch.from_numpy(bg_np).to(DEV)
    out = torch.empty((B, D, N), dtype=torch.float32, device=DEV)
    ws = gen.alloc_workspace(B)
    _say("oversampled ext_k=%d" % ext_k)
    gen.generate_batch_oversampled(8, 3, B, ext_k, bg, out, ws)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    params, offs = params.cpu().numpy(), offs.cpu().numpy()
    p, o = priors.sample_params(cfg, 8, 3 * B, B, bg_np.shape[1], ext_k=ext_k)
    np.testing.assert_allclose(params, p, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(offs, o)
    g = out.cpu().numpy()
    for i in range(0, B, 3):
        ref = pipeline.generate_sample(cfg, bg_np, p[:, i], int(o[i]))
        for d in range(D):
            assert rel_l2(g[i, d], ref[d]) <= 1e-5, (i, d)
    if ext_k == 1:
        plain = torch.empty_like(out)
        gen.generate_batch(8, 3, B, bg, plain, gen.alloc_workspace(B))
        torch.cuda.synchronize()
        assert torch.equal(plain, out)


def test_oversampling_rejects_bad_k():
    cfg = inputs.config("pr1_plain")
    gen = gwgen.Generator(cfg)
    bg = torch.zeros((2, 1 << 20), dtype=torch.float32, device=DEV)
    out = torch.empty((2, 2, gen.sizes["N"]), dtype=torch.float32, device=DEV)
    with pytest.raises(gwgen.GWError):
        gen.generate_batch_oversampled(1, 0, 2, 0, bg, out, gen.alloc_workspace(2))


@pytest.mark.parametrize("prec", [0, 2])
def test_view_pairs_in_other_precision_modes(prec):
    """The one-pass view-pair kernel in binary32 throughout (0) and binary64
    (2): the shifted view equals the plain batch bit for bit, and the
    reference view follows the oracle (mode 2 to the output's binary32
    rounding; mode 0 within the bound its binary32 phase allows)."""
    name = "paper_scale"
    cfg = inputs.config(name, precision=prec)
    bg_np = bg_for(name, 21)
    gen = gwgen.Generator(cfg)
    B, D, N = 4, gen.sizes["D"], gen.sizes["N"]
    bg = torch.from_numpy(bg_np).to(DEV)
    ref_t = torch.empty((B, D, N), dtype=torch.float32, device=DEV)
    shf_t = torch.empty_like(ref_t)
    ws = gen.alloc_workspace(B)
    _say("view pairs %s precision %d" % (name, prec))
    gen.generate_batch_pairs(6, 2, B, bg, ref_t, shf_t, ws)
    plain = torch.empty_like(ref_t)
    gen.generate_batch(6, 2, B, bg, plain, gen.alloc_workspace(B))
    torch.cuda.synchronize()
    assert torch.equal(shf_t, plain)
    p, o = priors.sample_params(cfg, 6, 2 * B, B, bg_np.shape[1])
    got = ref_t.cpu().numpy()
    worst = 0.0
    for i in range(B):
        d_ref, _ = pipeline.generate_pair(cfg, bg_np, p[:, i], int(o[i]))
        for d in range(D):
            worst = max(worst, rel_l2(got[i, d], d_ref[d]))
    _say("view pairs precision %d: reference view worst rel L2 %.3e" % (prec, worst))
    assert worst < (2e-7 if prec == 2 else 1e-2)
