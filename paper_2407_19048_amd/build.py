"""Build libgwgen.so in-tree for gfx950 with hipcc.

Each translation unit is compiled to an object file in its own hipcc
process (in parallel), then the objects are linked into the shared library.

    python -m paper_2407_19048_amd.build
"""

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC_NAMES = ("gwgen.hip", "gw_ragged.hip", "gw_long.hip", "gw_surrogate.hip")
SRCS = [os.path.join(_HERE, "csrc", n) for n in SRC_NAMES]
OUT = os.path.join(_HERE, "libgwgen.so")
OBJ_DIR = os.path.join(os.path.dirname(_HERE), "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose=True):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs, procs = [], []
    for src in SRCS:
        obj = os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(src))[0] + ".o")
        cmd = [hipcc] + HIPCC_FLAGS + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    failed = []
    for src, p in zip(SRCS, procs):
        text, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(text)
            failed.append((os.path.basename(src), p.returncode))
    if failed:
        raise RuntimeError("hipcc failed: %s" % ", ".join("%s (status %d)" % f for f in failed))
    tmp = OUT + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed with status %d" % r.returncode)
    os.replace(tmp, OUT)
    return OUT


def build_host_sanitized(out, verbose=False):
    """The library with its host side built with AddressSanitizer and
    UndefinedBehaviorSanitizer (device code unsanitized, at -O1), for
    checking the host-side argument validation and bookkeeping on a machine
    without a GPU.  Loaded with the sanitizer runtime preloaded."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    flags = ["--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-Xarch_host", "-g"] + san
    objs, procs = [], []
    for src in SRCS:
        obj = os.path.join(OBJ_DIR, os.path.splitext(os.path.basename(src))[0] + ".asan.o")
        cmd = [hipcc] + flags + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for src, p in zip(SRCS, procs):
        text, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (os.path.basename(src), text))
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + san + ["-o", out] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    return out


if __name__ == "__main__":
    build()
