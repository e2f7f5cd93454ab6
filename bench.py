"""Throughput of the on-the-fly training-data generator on one MI355X.

A step is one whole batch of the paper-scale workload: 2048 samples, three
detectors (H1, L1, V1), 8 s windows at 2048 Hz, IMR-form waveforms, a Welch
PSD per (sample, detector) from the 64 s of background preceding its window.
Steps run back to back on the resident background (2^27 samples per detector)
with every input already in HBM; the timed steps are replays of the captured
batch graph after the radix-order autotuner has run.  Also reported: the same
steps issued eagerly, the surrogate path, and the uneven workload (16384
signals over six (rate, duration) classes, one persistent launch per stage).
Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "whitened 3-det 8s@2048Hz samples/sec (plain vs surrogate) + % HBM roofline"
HBM_PEAK_GBS = 8000.0
# binary32 vector peak without packed instructions (the library is compiled
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
VALU_PEAK_PACKED_TFLOPS = 157.3


def log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


# ------------------------------------------------------------ CPU baseline

def _oracle_worker(args):
    cfg, slices, params, budget_s = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np  # noqa: F401
    import oracle
    done, t0 = 0, time.perf_counter()
    while True:
        for bg, p in zip(slices, params):
            oracle.generate_sample(cfg, bg, p, 0)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                return done, time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """(cores this process may run on, cores the host reports)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return usable, os.cpu_count() or usable


def cpu_baseline(cfg, bg, seed, B, budget_s, workers, one_core_s):
    """The FP64 oracle on the same workload: `workers` single-threaded
    processes, each regenerating its share of a fixed sample set until the
    time budget; then one process alone for the one-core figure."""
    import numpy as np
    import oracle
    z = oracle.derived_sizes(cfg)
    n_distinct = min(B, 4 * workers)
    params, offs = oracle.sample_params(cfg, seed, 0, n_distinct, bg.shape[1])
    slices = [np.ascontiguousarray(bg[:, o:o + z["P"] + z["N"]]) for o in offs]
    jobs = []
    for w in range(workers):
        sel = list(range(w, n_distinct, workers))
        jobs.append((cfg, [slices[i] for i in sel], [params[:, i] for i in sel], budget_s))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, jobs)
        one = pool.apply(_oracle_worker, ((cfg, slices[:4], [params[:, i] for i in range(4)], one_core_s),))
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    usable, reported = host_cores()
    return dict(value=done / busy, unit="samples/s", cores=workers, kind="oracle",
                one_core=round(one[0] / one[1], 2), host_cores_usable=usable, host_cores_reported=reported,
                cpu_model=cpu_model(),
                sample="%d oracle samples (FP64 NumPy, %d distinct draws of the paper-scale "
                       "workload) over %.1f s in %d processes, one thread each, then %d samples "
                       "in one process alone over %.1f s; %.1f s wall with start-up"
                       % (done, n_distinct, busy, workers, one[0], one[1], wall))


# --------------------------------------------------------- surrogate leg

def surrogate_leg(gen, bg, args, K, W, dev):
    """Learned-surrogate path at batch 8192: train it on the GPU (setup, not
    timed), measure held-out mismatch against the plain model, then time the
    fused surrogate batch and the plain batch at the same size."""
    import numpy as np
    import torch
    from paper_2407_19048_amd import inputs
    from paper_2407_19048_amd import surrogate as GS
    B = args.surrogate_batch
    z = gen.sizes
    f = np.arange(z["F"]) / gen.cfg["t_window"]
    psd = torch.from_numpy(inputs.true_psd(f, gen.cfg["fs"]).astype(np.float32)).to(dev)
    t0 = time.perf_counter()
    s = GS.Surrogate(gen, max_batch=8192)
    n_train, n_basis = 1 << 20, 32768
    fit = s.fit(seed=3, n_basis=n_basis, n_train=n_train, epochs=40, batch=8192, lr=2e-3, weight_decay=2e-3,
                n_head=8192, psd=psd)
    t_fit = time.perf_counter() - t0
    log("surrogate trained in %.1f s (mse %.3f -> %.3f)" % (t_fit, fit["initial_mse"], fit["final_mse"]))
    # held-out mismatch
    p = torch.empty((12, 8192), dtype=torch.float64, device=dev)
    o = torch.empty(8192, dtype=torch.int64, device=dev)
    gen.sample_params(4, 1 << 41, 8192, z["P"] + z["N"], p, o)
    mm, logmm, mm_max = s.mismatch_vs_plain(p, psd, maximised=True)
    mm = mm.cpu().numpy()
    mm_max = mm_max.cpu().numpy()
    fb = ~(logmm.cpu().numpy() <= -3.0)
    # what the network adds: the same state with its output layer zeroed
    # (coefficients from the linear skip path alone)
    s_lin = GS.Surrogate(gen, max_batch=8192)
    s_lin.set_state(*s.get_state())
    flat = s.get_weights()
    flat[sum(a * b + b for a, b in GS.LAYERS[:-1]):] = 0.0
    s_lin.set_weights(flat)
    mm_lin = s_lin.mismatch_vs_plain(p, psd)[0].cpu().numpy()
    s_lin.close()
    # waveform stage alone, same draws
    hp = torch.empty((8192, z["F"]), dtype=torch.complex64, device=dev)
    hc = torch.empty_like(hp)
    nodes = torch.empty((8192, 2, 1024), dtype=torch.float32, device=dev)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    gen.gen_fd_waveform(p, hp, hc)
    s.nodes(p, nodes)
    s.waveform(p, nodes, hp, hc)
    e[0].record()
    for _ in range(5):
        gen.gen_fd_waveform(p, hp, hc)
    e[1].record()
    for _ in range(5):
        s.nodes(p, nodes)
        s.waveform(p, nodes, hp, hc)
    e[2].record()
    torch.cuda.synchronize()
    wf_plain, wf_surr = e[0].elapsed_time(e[1]) / 5, e[1].elapsed_time(e[2]) / 5
    del hp, hc, nodes
    # whole batch, surrogate vs plain at B
    out = torch.empty((B, z["D"], z["N"]), dtype=torch.float32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    ws_s = gen.alloc_workspace_surrogate(B, device=dev)
    ws_p = gen.alloc_workspace(B, device=dev)
    timing = {}
    fallback_rate = 0.0
    for name in ("surrogate", "plain"):
        for i in range(W):
            if name == "surrogate":
                gen.generate_batch_surrogate(s, 5, i, B, bg, out, ws_s, status=status)
            else:
                gen.generate_batch(5, i, B, bg, out, ws_p, status=status)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(K):
            if name == "surrogate":
                gen.generate_batch_surrogate(s, 5, W + i, B, bg, out, ws_s, status=status)
            else:
                gen.generate_batch(5, W + i, B, bg, out, ws_p, status=status)
        torch.cuda.synchronize()
        timing[name] = (time.perf_counter() - t1) / K
        if name == "surrogate":
            fallback_rate = float(((status.cpu().numpy() & 16) != 0).mean())
    del out, ws_s, ws_p
    return {
        "batch": B,
        "value": round(B / timing["surrogate"], 1),
        "plain_value_same_batch": round(B / timing["plain"], 1),
        "end_to_end_gain": round(timing["plain"] / timing["surrogate"], 4),
        "ms_per_step": round(1e3 * timing["surrogate"], 4),
        "waveform_stage_ms": {"plain": round(wf_plain, 4), "surrogate": round(wf_surr, 4),
                              "gain": round(wf_plain / wf_surr, 3)},
        "mismatch_heldout": {"n": 8192, "median": float(np.median(mm)), "p90": float(np.percentile(mm, 90)),
                             "median_after_fallback": float(np.median(np.where(fb, 0.0, mm))),
                             "median_skip_path_only": float(np.median(mm_lin)),
                             "maximised": {"median": float(np.median(mm_max)),
                                           "p90": float(np.percentile(mm_max, 90))}},
        "training": {"n_train": n_train, "n_basis": n_basis, "weight_decay": fit["weight_decay"],
                     "initial_mse": round(fit["initial_mse"], 4), "final_mse": round(fit["final_mse"], 4)},
        "fallback_rate": round(fallback_rate, 4),
        "train_seconds": round(t_fit, 2),
        "train_steps": fit["steps"],
    }


# ------------------------------------------------------------------- main

# What the paper reports for its own pipeline (other hardware, other shapes):
# context for the figures above, not a like-for-like target.
PAPER_CONTEXT = {
    "waveform_generation": "about 0.15 s per 1000 waveforms on an NVIDIA A40 (section 3.2; IMRPhenomD, "
                           "two detectors, 4 s at 2048 Hz, waveform step only)",
    "training_throughput": "about 32 M simulations in 20-24 h on one A40 or A100 40 GB, i.e. 370-440 "
                           "samples/s including the network's forward and backward passes (section 5.1)",
    "online_latency": "about 6 s from data acquisition to posteriors and skymaps for the search plus "
                      "parameter estimation (abstract, section 7)",
}


def long_leg(bg, args, K, W, dev):
    """Long-duration binary neutron stars: 256 s windows at 2048 Hz (N = 2^19),
    batch 256; the window transforms run as four-step FFTs through HBM."""
    import torch
    from paper_2407_19048_amd import gwgen, inputs
    cfg = inputs.config("bns_long", precision=args.precision)
    gen = gwgen.Generator(cfg)
    z = gen.sizes
    B = cfg["batch"]
    out = torch.empty((B, z["D"], z["N"]), dtype=torch.float32, device=dev)
    ws = gen.alloc_workspace(B, device=dev)
    gen.autotune(B, bg, out, ws, reps=2)
    graph = gen.graph(2, 0, B, bg, out, ws)
    for _ in range(W):
        graph.launch()
    torch.cuda.synchronize()
    Kl = max(1, K // 5)
    t0 = time.perf_counter()
    for _ in range(Kl):
        graph.launch()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    graph.close()
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("non-finite long-window output")
    nbytes = B * z["D"] * (z["P"] + 2 * z["N"]) * 4
    gbs = nbytes / (el / Kl) / 1e9
    log("long windows: %.3f ms/batch of %d, %.0f samples/s, %.0f GB/s algorithmic"
        % (1e3 * el / Kl, B, B * Kl / el, gbs))
    return {"workload": "long-duration BNS: batch %d, 256 s windows at 2048 Hz (N = 2^19), TaylorF2, "
                        "Welch over the preceding 64 s" % B,
            "value": round(B * Kl / el, 1), "unit": "samples/s", "ms_per_step": round(1e3 * el / Kl, 4),
            "steps": Kl, "hbm_frac_algorithmic": round(gbs / HBM_PEAK_GBS, 4)}


def burst_leg(bg, args, K, W, dev):
    """Sine-Gaussian bursts at the paper-scale shape (same background, Welch
    and whitening; the waveform family changes)."""
    import torch
    from paper_2407_19048_amd import gwgen, inputs
    cfg = inputs.config("sine_gaussian", precision=args.precision)
    gen = gwgen.Generator(cfg)
    z = gen.sizes
    B = args.batch
    out = torch.empty((B, z["D"], z["N"]), dtype=torch.float32, device=dev)
    ws = gen.alloc_workspace(B, device=dev)
    gen.autotune(B, bg, out, ws, reps=2)
    graph = gen.graph(2, 0, B, bg, out, ws)
    for _ in range(W):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        graph.launch()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    graph.close()
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("non-finite burst output")
    log("sine-Gaussian: %.3f ms/batch, %.0f samples/s" % (1e3 * el / K, B * K / el))
    return {"workload": "sine-Gaussian bursts, paper-scale shape (f0 32-1000 Hz, Q 3-30, hrss 1e-23-1e-21)",
            "value": round(B * K / el, 1), "unit": "samples/s", "ms_per_step": round(1e3 * el / K, 4)}


def pairs_leg(gen, bg, args, K, W, dev):
    """View pairs (reference and shifted view of every sample) at the
    paper-scale shape: one prior draw and one Welch PSD per pair."""
    import torch
    z = gen.sizes
    B, D, N = args.batch, z["D"], z["N"]
    ref = torch.empty((B, D, N), dtype=torch.float32, device=dev)
    shf = torch.empty_like(ref)
    ws = gen.alloc_workspace(B, device=dev)
    for i in range(W):
        gen.generate_batch_pairs(2, i, B, bg, ref, shf, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        gen.generate_batch_pairs(2, W + i, B, bg, ref, shf, ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nbytes = B * D * (z["P"] + N + 2 * N) * 4
    log("view pairs: %.3f ms/batch, %.0f pairs/s" % (1e3 * el / K, B * K / el))
    return {"workload": "paper_scale view pairs (reference view at t_ref = T - 1.5 s and the shifted view)",
            "value": round(B * K / el, 1), "unit": "pairs/s", "ms_per_step": round(1e3 * el / K, 4),
            "hbm_frac_algorithmic": round(nbytes / (el / K) / 1e9 / HBM_PEAK_GBS, 4)}


def runpsd_leg(gen, bg, args, K, W, dev):
    """Per-run PSD mode at the paper-scale shape: one Welch PSD per detector
    over the whole background, a truncated whitening filter (fduration 2 s),
    then batches that only generate, inject and whiten (2 s cropped)."""
    import torch
    z = gen.sizes
    B, D, N = args.batch, z["D"], z["N"]
    fs = gen.cfg["fs"]
    M = int(round(2.0 * fs))
    crop = M // 2
    stride = z["K"] * (z["L"] // 2)
    n_chunks = (int(bg.shape[1]) - z["P"]) // stride + 1
    psd = torch.empty((D, z["Fw"]), dtype=torch.float32, device=dev)
    filt = torch.empty((D, z["F"]), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ws_psd = gen.run_psd(bg, n_chunks, psd)
    gen.whiten_filter(psd, M, filt)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    del ws_psd
    out = torch.empty((B, D, N - 2 * crop), dtype=torch.float32, device=dev)
    ws = gen.alloc_workspace(B, device=dev)
    for i in range(W):
        gen.generate_batch_runpsd(2, i, B, bg, filt, crop, out, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        gen.generate_batch_runpsd(2, W + i, B, bg, filt, crop, out, ws)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("non-finite per-run output")
    nbytes = B * D * (N + (N - 2 * crop)) * 4
    gbs = nbytes / (el / K) / 1e9
    log("per-run PSD: %.3f ms/batch, %.0f samples/s, %.0f GB/s algorithmic; setup %.1f ms (%d Welch chunks)"
        % (1e3 * el / K, B * K / el, gbs, setup_ms, n_chunks))
    return {
        "workload": "paper_scale shape, one Welch PSD per detector over the whole background (%d x 64 s), "
                    "truncated whitening filter (fduration 2 s), 1 s cropped at each end" % n_chunks,
        "value": round(B * K / el, 1), "unit": "samples/s", "ms_per_step": round(1e3 * el / K, 4),
        "hbm_frac_algorithmic": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_step": nbytes,
        "output_samples_per_window": N - 2 * crop, "setup_ms": round(setup_ms, 2),
    }


def ragged_leg(bg2048, args, K, W, dev):
    """Uneven workload: 16384 signals, (fs, T) in {1024, 2048} Hz x {4, 8, 16} s,
    classes drawn uniformly; the 2048 Hz classes share the main background,
    the 1024 Hz classes use one of 2^26 samples per detector."""
    import numpy as np
    import torch
    from paper_2407_19048_amd import gwgen, inputs
    classes = inputs.ragged_classes(precision=args.precision)
    t0 = time.perf_counter()
    bg1024 = torch.from_numpy(inputs.background(3, 1 << (args.log2_bg - 1), 1024.0, seed=3)).to(dev)
    log("ragged: 1024 Hz background in %.1f s" % (time.perf_counter() - t0))
    bgs = [bg1024 if c["fs"] == 1024.0 else bg2048 for c in classes]
    Br = args.ragged_batch
    cls = inputs.ragged_assignment(Br)
    rg = gwgen.Ragged(classes, cls)
    out = rg.alloc_out(device=dev)
    ws = rg.alloc_workspace(device=dev)
    pf = torch.empty((12, Br), dtype=torch.float32, device=dev)
    st = torch.empty(Br, dtype=torch.int32, device=dev)
    table = rg.autotune(bgs, out, ws, reps=3)
    tuned = {"ord_window": rg.get_tuning(gwgen.RTUNE_ORD_WINDOW), "ord_welch": rg.get_tuning(gwgen.RTUNE_ORD_WELCH),
             "grid_window": rg.get_tuning(gwgen.RTUNE_GRID_WINDOW),
             "grid_welch": rg.get_tuning(gwgen.RTUNE_GRID_WELCH),
             "window_mode": rg.get_tuning(gwgen.RTUNE_WINDOW_MODE),
             "welch_mode": rg.get_tuning(gwgen.RTUNE_WELCH_MODE)}
    log("ragged autotune %s -> %s" % (table, tuned))
    graph = rg.graph(2, 0, bgs, out, ws, params_f32=pf, status=st)
    for _ in range(W):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        graph.launch()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("non-finite ragged output")
    Ke = min(K, 10)
    t0 = time.perf_counter()
    for i in range(Ke):
        rg.generate(2, W + i, bgs, out, ws, pf, st)
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0) / Ke
    graph.close()
    # algorithmic bytes: D (P + N) read and D N written per signal
    nbytes = 0
    for c, n in zip(classes, np.bincount(cls, minlength=len(classes))):
        P, N = int(c["psd_length"] * c["fs"]), int(c["t_window"] * c["fs"])
        nbytes += int(n) * 3 * (P + 2 * N) * 4
    ms = 1e3 * el / K
    gbs = nbytes / (el / K) / 1e9
    welch_best = min(list(table["welch"].values()) + list(table["welch_class"].values()))
    win_best = min(table["window"].values())
    log("ragged: %.3f ms/batch, %.0f samples/s, %.0f GB/s algorithmic" % (ms, Br / (el / K), gbs))
    return {
        "workload": "uneven: %d signals, H1+L1+V1, (fs, T) uniform over {1024, 2048} Hz x {4, 8, 16} s, "
                    "Welch over the 64 s before each window" % Br,
        "value": round(Br * K / el, 1), "unit": "samples/s", "ms_per_step": round(ms, 4),
        "eager_ms_per_step": round(eager_ms, 4), "hbm_frac_algorithmic": round(gbs / HBM_PEAK_GBS, 4),
        "bytes_per_step": nbytes, "class_counts": np.bincount(cls, minlength=len(classes)).tolist(),
        "stage_ms": {"welch": round(welch_best, 4), "window": round(win_best, 4)},
        "autotune_ms": {"welch_ord%d_grid%d" % k: round(v, 4) for k, v in table["welch"].items()}
        | {"window_mode%d_ord%d" % k: round(v, 4) for k, v in table["window"].items()}
        | {"welch_per_class_ord%d" % k: round(v, 4) for k, v in table["welch_class"].items()},
        "tuned": tuned,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--log2-bg", type=int, default=27)
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle processes of the CPU baseline (at most the usable cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-batch", type=int, default=8192)
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-runpsd", action="store_true")
    ap.add_argument("--no-pairs", action="store_true")
    ap.add_argument("--no-burst", action="store_true")
    ap.add_argument("--no-long", action="store_true")
    ap.add_argument("--ragged-batch", type=int, default=16384)
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="after the timed region, copy a buffer of this size three times "
                         "(calibrates HBM byte counters against a known transfer)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this generator has no cross-GPU step "
              "(samples are independent), so a run on N GPUs is N independent copies of this one",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2407_19048_amd import inputs

    cfg = inputs.config("paper_scale", precision=args.precision)
    B, K, W = args.batch, args.steps, args.warmup
    n_det = len(cfg["det_ids"])
    t0 = time.perf_counter()
    bg_np = inputs.background(n_det, 1 << args.log2_bg, cfg["fs"], seed=1)
    log("background %s generated in %.1f s" % (bg_np.shape, time.perf_counter() - t0))

    cpu = None
    if not args.no_cpu_baseline:
        # every core this process may use, up to the host's share per GPU
        # (16 on the GPU hosts this runs on)
        workers = max(1, min(args.cpu_workers, host_cores()[0]))
        cpu = cpu_baseline(cfg, bg_np, 2, B, args.cpu_budget, workers, args.cpu_budget / 2)
        log("cpu baseline: %.1f samples/s on %d cores (%.1f on one core; %s, %d usable of %d reported)"
            % (cpu["value"], cpu["cores"], cpu["one_core"], cpu["cpu_model"], cpu["host_cores_usable"],
               cpu["host_cores_reported"]))

    import numpy as np
    import torch
    from paper_2407_19048_amd import gwgen
    gwgen.lib()
    dev = torch.device("cuda:0")
    bg = torch.from_numpy(bg_np).to(dev)
    del bg_np
    gen = gwgen.Generator(cfg)
    z = gen.sizes
    out = torch.empty((B, n_det, z["N"]), dtype=torch.float32, device=dev)
    pf = torch.empty((12, B), dtype=torch.float32, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    ws = gen.alloc_workspace(B, device=dev)
    seed = 2

    tune = gen.autotune(B, bg, out, ws, reps=3)
    tuned = {"ord_window": gen.get_tuning(gwgen.TUNE_ORD_WINDOW), "ord_welch": gen.get_tuning(gwgen.TUNE_ORD_WELCH),
             "occ_welch": gen.get_tuning(gwgen.TUNE_OCC_WELCH)}
    log("autotune %s -> %s" % (tune, tuned))
    graph = gen.graph(seed, 0, B, bg, out, ws, params_f32=pf, status=status)
    for i in range(W):
        graph.launch()
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    for i in range(K):
        graph.launch()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("timed %d graph steps in %.3f s" % (K, elapsed))
    value = B * K / elapsed
    ms_step = 1e3 * elapsed / K
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("non-finite output")
    # per-replay times with events around each graph launch (outside the
    # timed region): median and spread of single batches
    pairs_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for e0, e1 in pairs_ev:
        e0.record()
        graph.launch()
        e1.record()
    torch.cuda.synchronize()
    per_ms = np.array([e0.elapsed_time(e1) for e0, e1 in pairs_ev])
    log("graph replay events: median %.4f ms, p10 %.4f, p90 %.4f over %d replays"
        % (np.median(per_ms), np.percentile(per_ms, 10), np.percentile(per_ms, 90), K))
    # the same batches issued eagerly (three launches per step), for comparison
    Ke = min(K, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(Ke):
        gen.generate_batch(seed, W + i, B, bg, out, ws, pf, status)
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0) / Ke
    graph.close()

    # dominant kernel: segmented Welch, timed on its own with HIP events on the
    # stream the library launches on (torch's current stream)
    _, offs = gen.workspace_views(ws, B)
    psd = torch.empty((B, n_det, z["Fw"]), dtype=torch.float32, device=dev)
    for _ in range(2):
        gen.welch_psd(bg, offs, psd)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(K):
        gen.welch_psd(bg, offs, psd)
    ev1.record()
    torch.cuda.synchronize()
    welch_ms = ev0.elapsed_time(ev1) / K
    # algorithmic bytes per launch: every sample reads its P-sample stretch in
    # each detector once and writes its PSD
    welch_bytes = B * n_det * (z["P"] + z["Fw"]) * 4
    welch_gbs = welch_bytes / (welch_ms * 1e-3) / 1e9
    # algorithmic flops per launch: K segments of L per (sample, detector), a
    # real L-point FFT counted 2.5 L log2 L, plus window (L) and |X|^2 with
    # accumulation (2 L)
    L = z["L"]
    welch_flops = B * n_det * z["K"] * (2.5 * L * math.log2(L) + 3.0 * L)
    welch_tflops = welch_flops / (welch_ms * 1e-3) / 1e12
    from paper_2407_19048_amd.profiling import measured_traffic
    traffic = measured_traffic("k_welch", "paper_scale_B%d" % B)
    # the fused window kernel (second kernel of the step), timed by the
    # autotuner with events on its stream: per (sample, detector) it reads the
    # N-sample window and the Fw-bin PSD and writes N samples
    win_ms = tune["window_ord%d" % tuned["ord_window"]]
    win_bytes = B * n_det * (2 * z["N"] + z["Fw"]) * 4
    win_gbs = win_bytes / (win_ms * 1e-3) / 1e9
    window_rec = {"kernel": "k_window", "ms_per_launch": round(win_ms, 4), "bytes_per_launch": win_bytes,
                  "achieved_gbs": round(win_gbs, 1), "hbm_frac": round(win_gbs / HBM_PEAK_GBS, 4),
                  "traffic": measured_traffic("k_window", "paper_scale_B%d" % B)}

    # device-to-device copy of 1 GiB (or --copy-probe-gib): the bandwidth a
    # plain streaming kernel reaches on this part, timed with events on the
    # current stream, and the known transfer that calibrates byte counters
    gib = args.copy_probe_gib if args.copy_probe_gib > 0 else 1.0
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * 4 * n / (ev0.elapsed_time(ev1) / 5 * 1e-3) / 1e9
    log("copy probe: %d bytes read + written per copy, %.0f GB/s" % (4 * n, copy_gbs))
    del src, dst

    window_rec["frac_of_copy"] = round(win_gbs / copy_gbs, 4)
    # whole step, algorithmic bytes per sample: D (P + N) reads + D N writes
    step_bytes = B * n_det * ((z["P"] + z["N"]) + z["N"]) * 4
    step_gbs = step_bytes / (elapsed / K) / 1e9
    log("step %.3f ms (%.0f GB/s algorithmic, %.1f %% of HBM peak); welch %.3f ms (%.0f GB/s)"
        % (ms_step, step_gbs, 100 * step_gbs / HBM_PEAK_GBS, welch_ms, welch_gbs))

    surrogate = None
    if not args.no_surrogate:
        surrogate = surrogate_leg(gen, bg, args, K, W, dev)

    runpsd = None
    if not args.no_runpsd:
        runpsd = runpsd_leg(gen, bg, args, K, W, dev)
    pairs = None
    if not args.no_pairs:
        pairs = pairs_leg(gen, bg, args, K, W, dev)
    burst = None
    if not args.no_burst:
        burst = burst_leg(bg, args, K, W, dev)
    longw = None
    if not args.no_long:
        longw = long_leg(bg, args, K, W, dev)

    ragged = None
    if not args.no_ragged:
        ragged = ragged_leg(bg, args, K, W, dev)

    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "paper_scale: batch 2048, H1+L1+V1, 8 s windows at 2048 Hz, IMR-form "
                        "waveforms, per-sample Welch PSD over 64 s (2 s Hann, 1 s overlap), "
                        "plain path",
            "global_batch": B, "window_samples": z["N"], "psd_stretch_samples": z["P"],
            "background_samples_per_det": int(bg.shape[1]), "precision_mode": args.precision,
            "path": "plain",
            "issue": "hip graph replay",
            "eager_ms_per_step": round(eager_ms, 4),
            "replay_event_ms": {"median": round(float(np.median(per_ms)), 4),
                                "p10": round(float(np.percentile(per_ms, 10)), 4),
                                "p90": round(float(np.percentile(per_ms, 90)), 4), "n": int(K)},
            "autotune_ms": {k: round(v, 4) for k, v in tune.items()},
            "tuned": tuned,
            "step_hbm_frac_algorithmic": round(step_gbs / HBM_PEAK_GBS, 4),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_welch",
            "achieved": round(welch_tflops, 2),
            "peak": round(VALU_PEAK_TFLOPS, 1),
            "unit": "TFLOP/s",
            "frac": round(welch_tflops / VALU_PEAK_TFLOPS, 4),
            "frac_vs_packed_peak": round(welch_tflops / VALU_PEAK_PACKED_TFLOPS, 4),
            "flops_per_launch": welch_flops,
            "ms_per_launch": round(welch_ms, 4),
            "hbm_achieved_gbs": round(welch_gbs, 1),
            "hbm_frac": round(welch_gbs / HBM_PEAK_GBS, 4),
            "copy_gbs": round(copy_gbs, 1),
            "hbm_frac_of_copy": round(welch_gbs / copy_gbs, 4),
            "step_achieved_gbs": round(step_gbs, 1),
            "step_frac_of_copy": round(step_gbs / copy_gbs, 4),
            "bytes_per_launch": welch_bytes,
            "traffic": traffic,
            "window_kernel": window_rec,
        },
        "cpu_baseline": cpu,
        "surrogate": surrogate,
        "ragged": ragged,
        "per_run_psd": runpsd,
        "view_pairs": pairs,
        "sine_gaussian": burst,
        "long_windows": longw,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
