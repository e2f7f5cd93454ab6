"""Uneven (ragged) batches, captured pipelines and the autotuners, through the
C ABI.

Ragged parity: every checked slot against the FP64 oracle (whitened strain
relative L2 per (slot, detector) <= 1e-5; PSD RMS of (gpu/oracle - 1) <=
1e-4; params relative error <= 1e-12, offsets exact, row 11 = class).  A
ragged slot also matches the plain batch kernel for its class.  Graph
replays reproduce the eager calls bit for bit.
"""

import math
import sys

import numpy as np
import pytest

from oracle import pipeline
from paper_2407_19048_amd import gwgen, inputs
from draws import checked_draws

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL_STRAIN = 1e-5
TOL_PSD = 1e-4
DEV = "cuda"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


_BG = {}


def bg_for(fs, log2):
    key = (fs, log2)
    if key not in _BG:
        _BG[key] = inputs.background(3, 1 << log2, fs, seed=3 if fs == 1024.0 else 1)
    return _BG[key]


def class_bgs(classes, log2):
    return [bg_for(c["fs"], log2) for c in classes]


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def run_ragged(classes, cls, seed, batch_index, bgs_np, tune=None):
    rg = gwgen.Ragged(classes, cls)
    if tune:
        for k, v in tune.items():
            rg.set_tuning(k, v)
    bgs = []
    cache = {}
    for b in bgs_np:
        if id(b) not in cache:
            cache[id(b)] = _gpu(b)
        bgs.append(cache[id(b)])
    out = rg.alloc_out()
    ws = rg.alloc_workspace()
    pf = torch.empty((12, rg.B), dtype=torch.float32, device=DEV)
    st = torch.zeros(rg.B, dtype=torch.int32, device=DEV)
    rg.generate(seed, batch_index, bgs, out, ws, params_f32=pf, status=st)
    torch.cuda.synchronize()
    params, offs, psd = rg.workspace_views(ws)
    return dict(rg=rg, out=out.cpu().numpy(), params=params.cpu().numpy(), offs=offs.cpu().numpy(),
                psd=psd.cpu().numpy(), pf=pf.cpu().numpy(), status=st.cpu().numpy(), bgs=bgs, ws=ws, outt=out)


def check_slots(classes, cls, seed, batch_index, bgs_np, r, slots):
    rg = r["rg"]
    po, oo = pipeline.ragged_draws(classes, cls, seed, batch_index, [b.shape[1] for b in bgs_np], slots)
    worst = 0.0
    for i in slots:
        c = int(cls[i])
        cfg = classes[c]
        np.testing.assert_allclose(r["params"][:, i], po[:, i], rtol=1e-12, atol=0)
        assert r["params"][11, i] == float(c)
        assert r["offs"][i] == oo[i]
        ref, stages = pipeline.generate_sample(cfg, bgs_np[c], po[:, i], int(oo[i]), return_stages=True)
        got = rg.signal(torch.from_numpy(r["out"]), i).numpy()
        assert got.shape == ref.shape
        z = pipeline.derived_sizes(cfg)
        for d in range(3):
            e = rel_l2(got[d], ref[d])
            worst = max(worst, e)
            assert e <= TOL_STRAIN, (i, c, d, e)
            a = int(rg.psd_offset[i]) + d * z["Fw"]
            gp = r["psd"][a:a + z["Fw"]]
            ratio = gp.astype(np.float64) / stages["psd"][d]
            rms = math.sqrt(np.mean((ratio - 1.0) ** 2))
            assert rms <= TOL_PSD, (i, c, d, rms)
    return worst


def _balanced(B, n=6, seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    cls = np.array([k % n for k in range(B)], dtype=np.int32)
    rng.shuffle(cls)
    return cls


@pytest.mark.parametrize("mode", [0, 1])
def test_ragged_all_classes_match_oracle(mode):
    classes = inputs.ragged_classes()
    cls = _balanced(18)
    bgs = class_bgs(classes, 19)
    _say("ragged parity: B=18, six classes, window mode %d" % mode)
    r = run_ragged(classes, cls, 7, 2, bgs, tune={gwgen.RTUNE_WINDOW_MODE: mode})
    worst = check_slots(classes, cls, 7, 2, bgs, r, list(range(18)))
    _say("ragged worst rel L2 %.3e" % worst)
    np.testing.assert_array_equal(r["pf"], r["params"].astype(np.float32))


def test_ragged_group_tails_and_unused_classes():
    classes = inputs.ragged_classes()
    bgs = class_bgs(classes, 19)
    # 3 slots of the smallest class: 9 window items = one full group of 8
    # sub-blocks and one group with 7 idle sub-blocks; 9 Welch items (L =
    # 2048, pairs) end on a single; classes 1..4 unused
    cls = np.array([0, 5, 0, 0], dtype=np.int32)
    _say("ragged tails: cls=%s" % cls.tolist())
    r = run_ragged(classes, cls, 11, 0, bgs)
    check_slots(classes, cls, 11, 0, bgs, r, [0, 1, 2, 3])
    # a single slot
    cls1 = np.array([2], dtype=np.int32)
    r1 = run_ragged(classes, cls1, 12, 9, bgs)
    check_slots(classes, cls1, 12, 9, bgs, r1, [0])


def test_ragged_slot_matches_plain_kernel():
    classes = inputs.ragged_classes()
    bgs = class_bgs(classes, 19)
    cls = _balanced(12, seed=8)
    r = run_ragged(classes, cls, 3, 1, bgs)
    for c in (1, 4):
        gen = gwgen.Generator(classes[c])
        B = len(cls)
        out = torch.empty((B, 3, gen.sizes["N"]), dtype=torch.float32, device=DEV)
        ws = gen.alloc_workspace(B)
        gen.generate_batch(3, 1, B, r["bgs"][c], out, ws)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        for i in np.nonzero(cls == c)[0]:
            got = r["rg"].signal(torch.from_numpy(r["out"]), i).numpy()
            # same per-item code and inputs: equal up to instruction scheduling
            assert rel_l2(got, o[i]) <= 1e-6, (c, i)


def test_ragged_status_nyquist_flag():
    classes = inputs.ragged_classes()
    bgs = class_bgs(classes, 19)
    cls = _balanced(60, seed=9)
    r = run_ragged(classes, cls, 21, 0, bgs)
    p = r["params"]
    eta = p[1] / (1.0 + p[1]) ** 2
    Ms = p[0] * eta ** -0.6 * 4.925490947641267e-06
    fs = np.array([classes[c]["fs"] for c in cls])
    want = (0.2 / Ms > 0.5 * fs)
    got = (r["status"] & gwgen.STATUS_CUT_AT_NYQUIST) != 0
    # the decision is taken in binary64 on both sides; only a tie could differ
    assert np.array_equal(got, want)
    assert want.any() and (~want).any()


def test_ragged_full_size_sampled():
    classes = inputs.ragged_classes()
    cls = inputs.ragged_assignment(inputs.RAGGED_BATCH)
    bgs = class_bgs(classes, 22)
    _say("ragged full size: B=%d" % len(cls))
    r = run_ragged(classes, cls, 1, 0, bgs)
    slots = []
    for c in range(6):
        idx = np.nonzero(cls == c)[0]
        slots += [int(idx[0]), int(idx[-1])]
    worst = check_slots(classes, cls, 1, 0, bgs, r, sorted(slots))
    _say("ragged full size worst rel L2 %.3e" % worst)
    assert np.isfinite(r["out"]).all()


def _rel_graph_check(make_eager, graph, out_g, n=3, first=5):
    """Replay n times with eager work between replays; each replay must
    equal the eager call of its batch index bit for bit."""
    for rep in range(n):
        graph.launch()
        torch.cuda.synchronize()
        got = out_g.cpu().numpy().copy()
        want = make_eager(first + rep)
        assert np.array_equal(got, want), rep
        # unrelated eager work on the same stream between replays
        x = torch.randn(1 << 16, device=DEV)
        (x * 2).sum().item()
    graph.set_batch(first)
    graph.launch()
    torch.cuda.synchronize()
    assert np.array_equal(out_g.cpu().numpy(), make_eager(first))


@pytest.mark.parametrize("mode", [0, 1])
def test_ragged_graph_replays_match_eager(mode):
    classes = inputs.ragged_classes()
    bgs_np = class_bgs(classes, 19)
    cls = _balanced(12, seed=4)
    rg = gwgen.Ragged(classes, cls)
    rg.set_tuning(gwgen.RTUNE_WINDOW_MODE, mode)
    bgs = [_gpu(b) for b in bgs_np]
    out_g, ws_g = rg.alloc_out(), rg.alloc_workspace()
    st_g = torch.zeros(rg.B, dtype=torch.int32, device=DEV)
    graph = rg.graph(13, 5, bgs, out_g, ws_g, status=st_g)
    out_e, ws_e = rg.alloc_out(), rg.alloc_workspace()

    def eager(bi):
        rg.generate(13, bi, bgs, out_e, ws_e)
        torch.cuda.synchronize()
        return out_e.cpu().numpy().copy()

    _rel_graph_check(eager, graph, out_g)
    graph.close()


def test_plain_graph_replays_match_eager():
    cfg = inputs.config("paper_scale")
    gen = gwgen.Generator(cfg)
    bg = _gpu(bg_for(2048.0, 19))
    B = 8
    out_g = torch.empty((B, 3, gen.sizes["N"]), dtype=torch.float32, device=DEV)
    ws_g = gen.alloc_workspace(B)
    pf_g = torch.empty((12, B), dtype=torch.float32, device=DEV)
    graph = gen.graph(17, 5, B, bg, out_g, ws_g, params_f32=pf_g)
    out_e = torch.empty_like(out_g)
    ws_e = gen.alloc_workspace(B)

    def eager(bi):
        gen.generate_batch(17, bi, B, bg, out_e, ws_e)
        torch.cuda.synchronize()
        return out_e.cpu().numpy().copy()

    _rel_graph_check(eager, graph, out_g)
    graph.close()


@pytest.mark.parametrize("name", ["pr1_plain", "paper_scale"])
def test_plain_kernel_variants_match_oracle(name):
    import oracle
    cfg = inputs.config(name)
    bg_np = inputs.background(len(cfg["det_ids"]), 1 << 20, cfg["fs"], seed=1)
    bg = _gpu(bg_np)
    B = 6
    for ow, ol, occ in ((1, 1, 2), (0, 1, 3), (1, 0, 3)):
        gen = gwgen.Generator(cfg)
        gen.set_tuning(gwgen.TUNE_ORD_WINDOW, ow)
        gen.set_tuning(gwgen.TUNE_ORD_WELCH, ol)
        gen.set_tuning(gwgen.TUNE_OCC_WELCH, occ)
        out = torch.empty((B, len(cfg["det_ids"]), gen.sizes["N"]), dtype=torch.float32, device=DEV)
        ws = gen.alloc_workspace(B)
        gen.generate_batch(5, 0, B, bg, out, ws)
        torch.cuda.synchronize()
        params, offs = gen.workspace_views(ws, B)
        p, o = checked_draws(cfg, 5, 0, params.cpu().numpy(), offs.cpu().numpy(), bg_np.shape[1])
        ref = oracle.generate_batch(cfg, bg_np, p, o)
        g = out.cpu().numpy()
        for i in range(B):
            for d in range(len(cfg["det_ids"])):
                assert rel_l2(g[i, d], ref[i, d]) <= TOL_STRAIN, (name, ow, ol, occ, i, d)


def test_autotuners_keep_results():
    import oracle
    cfg = inputs.config("paper_scale")
    bg_np = bg_for(2048.0, 19)
    bg = _gpu(bg_np)
    B = 16
    gen = gwgen.Generator(cfg)
    out = torch.empty((B, 3, gen.sizes["N"]), dtype=torch.float32, device=DEV)
    ws = gen.alloc_workspace(B)
    rep = gen.autotune(B, bg, out, ws, reps=2)
    _say("plain autotune: %s" % rep)
    assert all(v > 0 for v in rep.values())
    assert gen.get_tuning(gwgen.TUNE_ORD_WINDOW) in (0, 1)
    gen.generate_batch(2, 0, B, bg, out, ws)
    torch.cuda.synchronize()
    params, offs = gen.workspace_views(ws, B)
    p, o = checked_draws(cfg, 2, 0, params.cpu().numpy(), offs.cpu().numpy(), bg_np.shape[1], idx=range(4))
    ref = oracle.generate_batch(cfg, bg_np, p[:, :4], o[:4])
    g = out.cpu().numpy()
    for i in range(4):
        assert rel_l2(g[i], ref[i]) <= TOL_STRAIN

    classes = inputs.ragged_classes()
    bgs_np = class_bgs(classes, 19)
    cls = _balanced(24, seed=6)
    rg = gwgen.Ragged(classes, cls)
    bgs = [_gpu(b) for b in bgs_np]
    rout, rws = rg.alloc_out(), rg.alloc_workspace()
    table = rg.autotune(bgs, rout, rws, reps=2)
    _say("ragged autotune: %s" % table)
    assert all(v > 0 for v in table["welch"].values()) and all(v > 0 for v in table["window"].values())
    assert all(v > 0 for v in table["welch_class"].values())
    tuned = {k: rg.get_tuning(k) for k in (gwgen.RTUNE_ORD_WINDOW, gwgen.RTUNE_ORD_WELCH,
                                          gwgen.RTUNE_GRID_WINDOW, gwgen.RTUNE_GRID_WELCH,
                                          gwgen.RTUNE_WINDOW_MODE, gwgen.RTUNE_WELCH_MODE)}
    _say("ragged tuned: %s" % tuned)
    r = run_ragged(classes, cls, 4, 0, bgs_np, tune=tuned)
    check_slots(classes, cls, 4, 0, bgs_np, r, list(range(0, 24, 3)))


def test_launch_shape_invariance():
    """Launch shapes that only change how the same items are spread over
    workgroups give bitwise-identical results: the plain Welch kernel at 2 and
    3 waves per SIMD, the persistent ragged launches at every grid, and the
    per-class Welch launch.  A missing LDS barrier or a queue race would show
    up as a difference."""
    cfg = inputs.config("paper_scale")
    bg = _gpu(bg_for(2048.0, 19))
    B = 16
    outs = []
    for occ in (2, 3):
        gen = gwgen.Generator(cfg)
        gen.set_tuning(gwgen.TUNE_OCC_WELCH, occ)
        gen.set_tuning(gwgen.TUNE_ORD_WINDOW, 1)
        out = torch.empty((B, 3, gen.sizes["N"]), dtype=torch.float32, device=DEV)
        ws = gen.alloc_workspace(B)
        _say("plain batch, Welch at %d waves per SIMD" % occ)
        gen.generate_batch(3, 1, B, bg, out, ws)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])

    classes = inputs.ragged_classes()
    bgs_np = class_bgs(classes, 19)
    cls = _balanced(30, seed=8)
    ref = None
    for wm, gw, gv in ((0, 1, 1), (0, 2, 1), (0, 4, 2), (1, 1, 1)):
        _say("ragged batch, Welch mode %d grid %d, window grid %d" % (wm, gw, gv))
        r = run_ragged(classes, cls, 5, 2, bgs_np,
                       tune={gwgen.RTUNE_WELCH_MODE: wm, gwgen.RTUNE_GRID_WELCH: gw, gwgen.RTUNE_GRID_WINDOW: gv,
                             gwgen.RTUNE_WINDOW_MODE: 0, gwgen.RTUNE_ORD_WELCH: 0, gwgen.RTUNE_ORD_WINDOW: 1})
        if ref is None:
            ref = r
        else:
            assert np.array_equal(r["psd"], ref["psd"])
            assert np.array_equal(r["out"], ref["out"])


def test_ragged_rejects_bad_input():
    classes = inputs.ragged_classes()
    with pytest.raises(gwgen.GWError):
        gwgen.Ragged(classes, np.array([0, 6], dtype=np.int32))  # class out of range
    bad = [dict(classes[0]), dict(classes[1], dl=(50.0, 3100.0))]  # priors differ
    with pytest.raises(gwgen.GWError):
        gwgen.Ragged(bad, np.array([0, 1], dtype=np.int32))
    rg = gwgen.Ragged(classes[:2], np.array([0, 1], dtype=np.int32))
    short = torch.zeros((3, 1000), dtype=torch.float32, device=DEV)
    with pytest.raises(gwgen.GWError):
        rg.generate(1, 0, [short, short], rg.alloc_out(), rg.alloc_workspace())
    with pytest.raises(gwgen.GWError):
        rg.set_tuning(gwgen.RTUNE_GRID_WELCH, 0)
