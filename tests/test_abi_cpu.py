"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/gwgen.h declares, and rejects bad arguments on the host
before any HIP call."""

import ctypes
import os
import re

import pytest

from paper_2407_19048_amd import gwgen, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "gwgen.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gw_status|const char\*|int64_t)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_six_steps_and_batch():
    names = _declared_functions()
    for n in ("sample_params", "gen_fd_waveform", "project_detectors", "inject", "welch_psd",
              "whiten", "gw_generate_batch", "gw_create", "gw_destroy"):
        assert n in names
    assert set(names) == set(gwgen.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = gwgen.lib()
    for n in _declared_functions():
        assert hasattr(L, n), n


def test_strerror():
    L = gwgen.lib()
    assert L.gw_strerror(0) == b"ok"
    assert L.gw_strerror(-1) == b"invalid argument"
    assert L.gw_strerror(-3) == b"HIP error"


def test_config_struct_layout():
    # int32 n_det, int32[4], pad, 6 doubles, 2 int32, 8 doubles, 6 doubles
    assert ctypes.sizeof(gwgen.GWConfig) == 4 + 16 + 4 + 48 + 8 + 64 + 48
    assert gwgen.GWConfig.f0.offset == 4 + 16 + 4 + 48 + 8 + 64


def _create(cfg):
    c = gwgen.make_config(cfg)
    h = ctypes.c_void_p()
    s = gwgen.lib().gw_create(ctypes.byref(c), ctypes.byref(h))
    return s, h


@pytest.mark.parametrize("override", [
    dict(t_window=3.0),                 # N not a power of two
    dict(t_window=1.0),                 # N = 1024: below the shortest window transform
    dict(fs=1000.0),                    # N not a power of two
    dict(fftlen=1.0, overlap=0.5),      # L = 1024 below the minimum
    dict(overlap=0.5),                  # stride not L/2
    dict(psd_length=32.5),              # P - L not a multiple of the stride
    dict(det_ids=(0, 1, 2, 0, 1)),      # too many detectors
    dict(det_ids=(0, 7)),               # unknown detector
    dict(approximant=3),
    dict(precision=5),
    dict(q=(0.5, 1.5)),
    dict(chi=(-1.2, 0.9)),
    dict(mc=(-1.0, 10.0)),
    dict(f_min=600.0),                  # above Nyquist of 1024 Hz
])
def test_create_rejects_bad_config_on_host(override):
    cfg = inputs.config("pr1_plain", **override)
    s, h = _create(cfg)
    assert s == gwgen.GW_EINVAL
    assert not h.value


def test_double_precision_longest_window_unsupported():
    cfg = inputs.config("paper_scale", t_window=16.0, precision=2)
    s, _ = _create(cfg)
    assert s == gwgen.GW_EUNSUPPORTED


def test_null_context_rejected():
    L = gwgen.lib()
    null = ctypes.c_void_p(0)
    v = ctypes.c_int64()
    assert L.gw_query(null, 0, ctypes.byref(v)) == gwgen.GW_EINVAL
    assert L.sample_params(null, 1, 0, 4, 1 << 20, null, null, null) == gwgen.GW_EINVAL
    assert L.welch_psd(null, null, 1 << 20, null, 4, null, null) == gwgen.GW_EINVAL
    assert L.whiten(null, null, null, 4, null, null, null) == gwgen.GW_EINVAL
    assert L.gw_generate_batch(null, 1, 0, 4, null, 1 << 20, null, null, null, null, 0, null) == gwgen.GW_EINVAL
    assert L.gw_generate_batch_noalloc(null, 1, 0, 4, null, 1 << 20, null, null, null, null) == gwgen.GW_EINVAL
    assert L.gw_destroy(null) == gwgen.GW_OK


def test_workspace_must_be_contiguous_device_memory():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        gwgen._workspace_bytes(torch.empty(64, dtype=torch.float64))  # host memory
