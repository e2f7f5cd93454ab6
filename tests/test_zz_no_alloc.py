"""The allocation-free batch entry point (static device scratch area)
against gw_generate_batch with a caller workspace, through the C ABI: two
calls in a row, the second with a smaller batch, bitwise equal windows,
trainer parameters and status; the first also against the oracle; no
device memory taken by the call; batches beyond the area rejected."""

import sys

import numpy as np
import pytest

import oracle
from paper_2407_19048_amd import gwgen, inputs
from draws import checked_draws

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_workspace_entry_point():
    cfg = inputs.config("paper_scale")
    gen = gwgen.Generator(cfg)
    z = gen.sizes
    bg_np = inputs.background(3, 1 << 22, cfg["fs"], seed=1)
    bg = torch.from_numpy(bg_np).to(DEV)
    for B, batch in ((2048, 3), (24, 5)):
        _say("no-alloc batch B=%d index %d" % (B, batch))
        out_a = torch.full((B, 3, z["N"]), np.nan, dtype=torch.float32, device=DEV)
        pf_a = torch.zeros((12, B), dtype=torch.float32, device=DEV)
        st_a = torch.full((B,), -1, dtype=torch.int32, device=DEV)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        gen.generate_batch_noalloc(7, batch, B, bg, out_a, pf_a, st_a)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        out_b = torch.empty_like(out_a)
        pf_b = torch.empty_like(pf_a)
        st_b = torch.empty_like(st_a)
        ws = gen.alloc_workspace(B)
        gen.generate_batch(7, batch, B, bg, out_b, ws, pf_b, st_b)
        torch.cuda.synchronize()
        assert free1 == free0, (free0, free1)
        assert torch.equal(out_a, out_b)
        assert torch.equal(pf_a, pf_b)
        assert torch.equal(st_a, st_b)
        if B == 24:
            params, offs = gen.workspace_views(ws, B)
            P, O = checked_draws(cfg, 7, batch * B, params.cpu().numpy(), offs.cpu().numpy(), bg_np.shape[1],
                                 idx=(0, 11, 23))
            o = out_a.cpu().numpy()
            for i in (0, 11, 23):
                ref = oracle.generate_sample(cfg, bg_np, P[:, i], int(O[i]))
                for d in range(3):
                    e = np.linalg.norm(o[i, d] - ref[d]) / np.linalg.norm(ref[d])
                    assert e < 1e-5, (i, d, e)


def test_noalloc_rejects_batches_beyond_the_area():
    cfg = inputs.config("paper_scale")
    gen = gwgen.Generator(cfg)
    per = gen.workspace_size(1024) / 1024.0
    B = int(gwgen.SCRATCH_BYTES / per) + 64
    assert gen.workspace_size(B) > gwgen.SCRATCH_BYTES
    bg = torch.zeros((3, 1 << 20), dtype=torch.float32, device=DEV)
    out = torch.empty((1, 3, 8), dtype=torch.float32, device=DEV)   # never written: rejected on the host
    with pytest.raises(gwgen.GWError, match="scratch"):
        gen._check(gwgen.lib().gw_generate_batch_noalloc(gen._h, 1, 0, B, gwgen._ptr(bg), bg.shape[1],
                                                         gwgen._ptr(out), None, None, gwgen._stream()), "noalloc")
