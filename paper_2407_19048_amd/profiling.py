"""Summaries of rocprofv3 runs for the profiles/ folder.

    python -m paper_2407_19048_amd.profiling stats STATS_CSV TITLE "COMMAND"
        kernel time table (markdown) from a --kernel-trace --stats run
    python -m paper_2407_19048_amd.profiling counters COUNTER_DIR KERNEL_SUBSTR TITLE "COMMAND"
        per-dispatch means of every counter of a --pmc run for the matching kernels (markdown)
    python -m paper_2407_19048_amd.profiling traffic FETCH_DIR WRITE_DIR KERNEL VARIANT GRID WORKLOAD COPY_GIB "COMMAND"
        HBM traffic record (JSON in profiles/) as described below
    python -m paper_2407_19048_amd.profiling trace TRACE_CSV "FILTER[;FILTER...]" TITLE "COMMAND"
        per (kernel, grid, workgroup) dispatch count, average and median duration (markdown) from the
        kernel trace of a --kernel-trace run, for the dispatches matching any FILTER: a kernel-name
        substring, optionally followed by @GRID[|GRID...] (total work-items) to keep only those grids
    python -m paper_2407_19048_amd.profiling valu COUNTER_DIR KERNEL_SUBSTR[,KERNEL_SUBSTR...] TITLE "COMMAND"
        VALU issue, LDS bank-conflict and wait shares per kernel (markdown) from a --pmc run with
        SQ_INSTS_VALU SQ_WAVES SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE SQ_WAIT_ANY SQ_WAVE_CYCLES

HBM traffic of a kernel from two rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are taken in separate runs of
the same command, which also copies a device buffer of known size (bench.py
--copy-probe-gib).  Each counter is scaled by the factor that makes it read
the known size on that copy, so the result is in bytes moved between the
chip and HBM.  The summary is stored with a hash of the sources of the
kernel's translation unit (KERNEL_SOURCES); the benchmark reports it only
while the hash still matches.

VARIANT is a substring of the demangled kernel name that selects the
instantiation the benchmark times (other variants, e.g. the autotuner's
candidates, are excluded); GRID is its grid size in work-items.
"""

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2407_19048_amd", "csrc")


# Sources of the translation unit that defines each profiled kernel (the
# .hip file and every header it includes); a traffic record stays valid while
# these are unchanged.  Kernels not listed hash every source.
_PLAIN_TU = ("paper_2407_19048_amd/csrc/gwgen.hip", "paper_2407_19048_amd/csrc/gw_fft.hpp",
             "paper_2407_19048_amd/csrc/gw_physics.hpp", "paper_2407_19048_amd/csrc/gw_internal.hpp",
             "paper_2407_19048_amd/csrc/gw_items.hpp", "include/gwgen.h")
KERNEL_SOURCES = {"k_welch": _PLAIN_TU, "k_window": _PLAIN_TU}


def _all_sources():
    return tuple(sorted(os.path.join("paper_2407_19048_amd", "csrc", f) for f in os.listdir(SRC)
                        if f.endswith((".hip", ".hpp")))) + ("include/gwgen.h",)


def kernel_source_hash(kernel=None):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel] if kernel in KERNEL_SOURCES else _all_sources():
        h.update(f.encode())
        with open(os.path.join(os.path.dirname(os.path.dirname(SRC)), f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_path(kernel, workload):
    return os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))


def measured_traffic(kernel, workload):
    """Stored HBM bytes per launch, or None if absent or the sources changed."""
    path = traffic_path(kernel, workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash(kernel):
        return None
    return d.get("hbm_bytes_per_launch")


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % d)
    out = []
    for f in files:
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def _copy_value(rows, counter):
    """Counter reading of the largest copy dispatch (the probe)."""
    cands = [r for r in rows if r["Counter_Name"] == counter and "copy" in r["Kernel_Name"].lower()]
    if not cands:
        raise ValueError("no copy dispatch found for %s" % counter)
    big = max(int(r["Grid_Size"]) for r in cands)
    vals = [float(r["Counter_Value"]) for r in cands if int(r["Grid_Size"]) == big]
    return sum(vals) / len(vals)


def summarise(fetch_dir, write_dir, kernel, variant, grid, workload, copy_gib, command):
    copy_bytes = int(copy_gib * (1 << 30)) // 4 * 4
    fr, wr = _rows(fetch_dir), _rows(write_dir)
    match = lambda r: variant in r["Kernel_Name"] and int(r["Grid_Size"]) == int(grid)
    f = [float(r["Counter_Value"]) for r in fr if r["Counter_Name"] == "FETCH_SIZE" and match(r)]
    w = [float(r["Counter_Value"]) for r in wr if r["Counter_Name"] == "WRITE_SIZE" and match(r)]
    if not f or not w:
        raise ValueError("kernel %s not found in the counter runs" % kernel)
    f_kib, w_kib = sum(f) / len(f), sum(w) / len(w)
    cf = copy_bytes / (_copy_value(fr, "FETCH_SIZE") * 1024.0)
    cw = copy_bytes / (_copy_value(wr, "WRITE_SIZE") * 1024.0)
    rec = {
        "kernel": kernel,
        "variant": variant,
        "grid": int(grid),
        "workload": workload,
        "source_hash": kernel_source_hash(kernel),
        "sources": list(KERNEL_SOURCES.get(kernel, ("every kernel source",))),
        "dispatches": [len(f), len(w)],
        "fetch_kib_per_dispatch": round(f_kib, 3),
        "write_kib_per_dispatch": round(w_kib, 3),
        "copy_probe_bytes": copy_bytes,
        "fetch_scale": round(cf, 4),
        "write_scale": round(cw, 4),
        "fetch_bytes_per_launch": round(f_kib * 1024.0 * cf),
        "write_bytes_per_launch": round(w_kib * 1024.0 * cw),
        "hbm_bytes_per_launch": round(f_kib * 1024.0 * cf + w_kib * 1024.0 * cw),
        "command": command,
    }
    os.makedirs(os.path.dirname(traffic_path(kernel, workload)), exist_ok=True)
    with open(traffic_path(kernel, workload), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def _col(header, *names):
    low = {h.lower(): h for h in header}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError("none of %s in %s" % (names, header))


def stats_table(stats_csv, title, command, top=14):
    """Markdown table of the kernels of a rocprofv3 --stats run, by total time."""
    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    if not rows:
        raise ValueError("empty stats file %s" % stats_csv)
    h = list(rows[0].keys())
    name, calls = _col(h, "Name", "KernelName"), _col(h, "Calls")
    total, avg = _col(h, "TotalDurationNs", "TotalDuration"), _col(h, "AverageNs", "Average")
    rows.sort(key=lambda r: -float(r[total]))
    grand = sum(float(r[total]) for r in rows)
    out = ["# %s" % title, "", "Command (one MI355X):", "", "    %s" % command, "",
           "Source: `%s` (every dispatch of the run)." % os.path.basename(stats_csv), "",
           "| kernel | calls | average | total | share |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append("| `%s` | %s | %.4f ms | %.3f ms | %.2f %% |"
                   % (short_name(r[name]), r[calls], float(r[avg]) / 1e6, float(r[total]) / 1e6, 100.0 * float(r[total]) / grand))
    return "\n".join(out) + "\n"


def counters_table(counter_dir, kernel_substr, title, command):
    """Markdown table: per-dispatch mean of each counter for the kernels whose
    name contains kernel_substr (one line per kernel name and grid)."""
    rows = [r for r in _rows(counter_dir) if kernel_substr in r["Kernel_Name"]]
    if not rows:
        raise ValueError("no dispatch of %s in %s" % (kernel_substr, counter_dir))
    acc = {}
    for r in rows:
        key = (r["Kernel_Name"], int(r["Grid_Size"]))
        acc.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for v in acc.values() for c in v})
    out = ["# %s" % title, "", "Command (one MI355X):", "", "    %s" % command, "",
           "Per-dispatch means (dispatch count in brackets).", "",
           "| kernel | grid | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for (k, g), v in sorted(acc.items()):
        cells = ["%.4g (%d)" % (sum(v[c]) / len(v[c]), len(v[c])) if c in v else "" for c in names]
        out.append("| `%s` | %d | %s |" % (k, g, " | ".join(cells)))
    return "\n".join(out) + "\n"


def short_name(name):
    """Demangled kernel name without 'void', anonymous-namespace qualifiers
    and the argument list: k_welch<float, double, 4096, 0, 3>."""
    n = name.replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def trace_table(trace_csv, filters, title, command):
    """Markdown table per (kernel, grid, workgroup size) from a rocprofv3
    kernel trace: dispatches, average and median duration, sorted by total
    time.  filters: kernel-name substrings separated by ';' (names contain
    commas), each optionally with @GRID[|GRID...] (grid sizes in work-items)
    to keep only those."""
    flt = []
    for f in filters.split(";"):
        if not f:
            continue
        sub, _, grids = f.partition("@")
        flt.append((sub, {int(g) for g in grids.split("|")} if grids else None))
    with open(trace_csv) as fh:
        rows = list(csv.DictReader(fh))
    acc = {}
    for r in rows:
        name = r["Kernel_Name"]
        grid = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y", 1) or 1) * int(r.get("Grid_Size_Z", 1) or 1)
        if not any(sub in name and (keep is None or grid in keep) for sub, keep in flt):
            continue
        wg = int(r["Workgroup_Size_X"]) * int(r.get("Workgroup_Size_Y", 1) or 1) * int(r.get("Workgroup_Size_Z", 1) or 1)
        acc.setdefault((name, grid, wg), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    if not acc:
        raise ValueError("no matching dispatch in %s" % trace_csv)
    out = ["# %s" % title, "", "Command (one MI355X):", "", "    %s" % command, "",
           "Per (kernel, grid, workgroup) from `%s`:" % os.path.basename(trace_csv), "",
           "| kernel | grid (work-items) | workgroup | dispatches | average | median | total |",
           "|---|---|---|---|---|---|---|"]
    for (name, grid, wg), ms in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        ms_s = sorted(ms)
        med = ms_s[len(ms_s) // 2] if len(ms_s) % 2 else 0.5 * (ms_s[len(ms_s) // 2 - 1] + ms_s[len(ms_s) // 2])
        out.append("| `%s` | %d | %d | %d | %.4f ms | %.4f ms | %.3f ms |"
                   % (short_name(name), grid, wg, len(ms), sum(ms) / len(ms), med, sum(ms)))
    return "\n".join(out) + "\n"


# MI355X: 256 CUs x 4 SIMDs; a wave64 VALU instruction occupies a 16-lane
# SIMD for 4 cycles (unpacked binary32 or binary64) at the 2.4 GHz peak clock
N_SIMD, CYCLES_PER_VALU, CLOCK_HZ = 1024, 4, 2.4e9


def valu_table(counter_dir, kernel_substrs, title, command):
    """Markdown table per (kernel, grid): waves, VALU instructions per wave,
    mean dispatch duration, VALU issue estimate 4 SQ_INSTS_VALU / (1024 SIMDs
    x duration x 2.4 GHz), LDS conflict share SQ_LDS_BANK_CONFLICT /
    SQ_LDS_IDX_ACTIVE and wait share SQ_WAIT_ANY / SQ_WAVE_CYCLES.  Durations
    come from the dispatch timestamps of the counter run."""
    subs = [k for k in kernel_substrs.split(",") if k]
    rows = [r for r in _rows(counter_dir) if any(k in r["Kernel_Name"] for k in subs)]
    if not rows:
        raise ValueError("no dispatch of %s in %s" % (kernel_substrs, counter_dir))
    acc, dur = {}, {}
    for r in rows:
        key = (r["Kernel_Name"], int(r["Grid_Size"]))
        acc.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        if r.get("Start_Timestamp") and r.get("End_Timestamp"):
            dur.setdefault(key, {})[r.get("Dispatch_Id", r.get("Correlation_Id"))] = (
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)

    def mean(v, c):
        return sum(v[c]) / len(v[c]) if c in v and v[c] else float("nan")

    out = ["# %s" % title, "", "Command (one MI355X):", "", "    %s" % command, "",
           "Per dispatch (mean over dispatches; duration from the dispatch timestamps of the counter run). "
           "A wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles (unpacked binary32 or binary64), "
           "so the VALU issue estimate is 4 x SQ_INSTS_VALU / (1024 SIMDs x duration x 2.4 GHz): exact at the "
           "2.4 GHz peak engine clock with every instruction taking 4 cycles; a lower clock raises the true "
           "fraction, and a value near or just above 100 % means the kernel is at the issue limit. LDS conflict "
           "share = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE; wait share = SQ_WAIT_ANY / SQ_WAVE_CYCLES (waves "
           "stalled on s_waitcnt).", "",
           "| kernel | grid | dispatches | waves | VALU instructions per wave | duration | VALU issue (estimate) "
           "| LDS conflict share | wait share |",
           "|---|---|---|---|---|---|---|---|---|"]
    for (k, g), v in sorted(acc.items(), key=lambda kv: -mean(kv[1], "SQ_INSTS_VALU")):
        waves, valu = mean(v, "SQ_WAVES"), mean(v, "SQ_INSTS_VALU")
        ds = list(dur.get((k, g), {}).values())
        d = sum(ds) / len(ds) if ds else float("nan")
        issue = CYCLES_PER_VALU * valu / (N_SIMD * d * CLOCK_HZ) if ds else float("nan")
        conf = mean(v, "SQ_LDS_BANK_CONFLICT") / mean(v, "SQ_LDS_IDX_ACTIVE") if mean(v, "SQ_LDS_IDX_ACTIVE") else 0.0
        wait = mean(v, "SQ_WAIT_ANY") / mean(v, "SQ_WAVE_CYCLES") if mean(v, "SQ_WAVE_CYCLES") else float("nan")
        n = max(len(x) for x in v.values())
        out.append("| `%s` | %d | %d | %.0f | %.0f | %.4f ms | %.1f %% | %.1f %% | %.1f %% |"
                   % (short_name(k), g, n, waves, valu / waves if waves else float("nan"), d * 1e3, 100 * issue,
                      100 * conf, 100 * wait))
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    a = sys.argv[1:]
    if len(a) == 4 and a[0] == "stats":
        sys.stdout.write(stats_table(a[1], a[2], a[3]))
    elif len(a) == 5 and a[0] == "counters":
        sys.stdout.write(counters_table(a[1], a[2], a[3], a[4]))
    elif len(a) == 5 and a[0] == "trace":
        sys.stdout.write(trace_table(a[1], a[2], a[3], a[4]))
    elif len(a) == 5 and a[0] == "valu":
        sys.stdout.write(valu_table(a[1], a[2], a[3], a[4]))
    elif len(a) == 9 and a[0] == "traffic":
        print(json.dumps(summarise(a[1], a[2], a[3], a[4], int(a[5]), a[6], float(a[7]), a[8]), indent=1))
    else:
        sys.exit(__doc__)
