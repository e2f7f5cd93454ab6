"""Build libgwgen.so in-tree for gfx950 with hipcc.

    python -m paper_2407_19048_amd.build
"""

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(_HERE, "csrc", n) for n in ("gwgen.hip", "gw_ragged.hip", "gw_long.hip", "gw_surrogate.hip")]
OUT = os.path.join(_HERE, "libgwgen.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose=True):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed with status %d" % r.returncode)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
