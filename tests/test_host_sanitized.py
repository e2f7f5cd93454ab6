"""The library's host side under AddressSanitizer and UndefinedBehavior-
Sanitizer (a separate build, sanitizers on the host code only), on a
machine without a GPU:
every entry point's argument validation, the configuration checks and the
strings run in a child process with the sanitizer runtime preloaded; any
report fails the test."""

import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

CHILD = r'''
import ctypes
from paper_2407_19048_amd import gwgen, inputs
L = gwgen.lib()
assert L.gw_strerror(0) == b"ok" and L.gw_strerror(-4) == b"unsupported configuration"
null = ctypes.c_void_p(0)
v = ctypes.c_int64()
bad = [dict(t_window=3.0), dict(fftlen=1.0, overlap=0.5), dict(overlap=0.5), dict(psd_length=32.5),
       dict(det_ids=(0, 1, 2, 0, 1)), dict(det_ids=(0, 7)), dict(approximant=3), dict(precision=5),
       dict(q=(0.5, 1.5)), dict(chi=(-1.2, 0.9)), dict(mc=(-1.0, 10.0)), dict(f_min=600.0)]
for over in bad:
    c = gwgen.make_config(inputs.config("pr1_plain", **over))
    h = ctypes.c_void_p()
    assert L.gw_create(ctypes.byref(c), ctypes.byref(h)) == gwgen.GW_EINVAL and not h.value, over
c = gwgen.make_config(inputs.config("paper_scale", t_window=16.0, precision=2))
assert L.gw_create(ctypes.byref(c), ctypes.byref(ctypes.c_void_p())) == gwgen.GW_EUNSUPPORTED
assert L.gw_create(None, None) == gwgen.GW_EINVAL
assert L.gw_query(null, 0, ctypes.byref(v)) == gwgen.GW_EINVAL
assert L.gw_workspace_size(null, 4, ctypes.byref(v)) == gwgen.GW_EINVAL
assert L.sample_params(null, 1, 0, 4, 1 << 20, null, null, null) == gwgen.GW_EINVAL
assert L.gen_fd_waveform(null, null, 4, null, null, null) == gwgen.GW_EINVAL
assert L.project_detectors(null, null, null, null, 4, null, null) == gwgen.GW_EINVAL
assert L.inject(null, null, 1 << 20, null, null, 4, null, null) == gwgen.GW_EINVAL
assert L.welch_psd(null, null, 1 << 20, null, 4, null, null) == gwgen.GW_EINVAL
assert L.whiten(null, null, null, 4, null, null, null) == gwgen.GW_EINVAL
assert L.gw_generate_batch(null, 1, 0, 4, null, 1 << 20, null, null, null, null, 0, null) == gwgen.GW_EINVAL
assert L.gw_generate_batch_noalloc(null, 1, 0, 4, null, 1 << 20, null, null, null, null) == gwgen.GW_EINVAL
assert L.gw_surrogate_create(null, 64, ctypes.byref(ctypes.c_void_p())) == gwgen.GW_EINVAL
assert L.gw_surrogate_set_adam(null, 0.9, 0.999, 1e-8) == gwgen.GW_EINVAL
assert L.gw_surrogate_train_step(null, null, null, 4, ctypes.c_float(1e-3), ctypes.c_float(0.0), null, null) == gwgen.GW_EINVAL
assert L.gw_surrogate_n_weights() > 0
assert L.gw_destroy(null) == gwgen.GW_OK and L.gw_surrogate_destroy(null) == gwgen.GW_OK
cls = (ctypes.c_int32 * 4)(0, 1, 0, 1)
cfgs = (gwgen.GWConfig * 2)(gwgen.make_config(inputs.config("pr1_plain")),
                            gwgen.make_config(inputs.config("pr1_plain", precision=2)))
assert L.gw_ragged_create(cfgs, 2, ctypes.cast(cls, ctypes.c_void_p), 4, ctypes.byref(ctypes.c_void_p())) == gwgen.GW_EUNSUPPORTED
assert L.gw_ragged_create(cfgs, 0, ctypes.cast(cls, ctypes.c_void_p), 4, ctypes.byref(ctypes.c_void_p())) == gwgen.GW_EINVAL
print("host checks passed")
'''


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.mark.timeout(900)
def test_host_side_under_sanitizers(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    rt = _asan_runtime()
    if not (os.path.exists(hipcc) or shutil.which("hipcc")) or rt is None:
        pytest.skip("hipcc or the clang sanitizer runtime is not available")
    from paper_2407_19048_amd import build
    lib = build.build_host_sanitized(str(tmp_path / "libgwgen_san.so"))
    env = dict(os.environ, GWGEN_LIB=lib, LD_PRELOAD=rt, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", CHILD], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "host checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
