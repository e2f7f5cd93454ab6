"""HBM traffic of a kernel from two rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are taken in separate runs of
the same command, which also copies a device buffer of known size (bench.py
--copy-probe-gib).  Each counter is scaled by the factor that makes it read
the known size on that copy, so the result is in bytes moved between the
chip and HBM.  The summary is stored with a hash of the kernel sources; the
benchmark reports it only while the hash still matches.

    python -m paper_2407_19048_amd.profiling FETCH_DIR WRITE_DIR KERNEL VARIANT GRID WORKLOAD COPY_GIB "COMMAND"

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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(SRC)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(SRC, f), "rb") as fh:
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
    if d.get("source_hash") != kernel_source_hash():
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
        "source_hash": kernel_source_hash(),
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


if __name__ == "__main__":
    a = sys.argv[1:]
    if len(a) != 8:
        sys.exit(__doc__)
    print(json.dumps(summarise(a[0], a[1], a[2], a[3], int(a[4]), a[5], float(a[6]), a[7]), indent=1))
