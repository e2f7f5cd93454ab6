"""ctypes binding of libgwgen.so (C ABI in include/gwgen.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Arrays are PyTorch device tensors; the library sees raw device pointers and
the current HIP stream.  Shapes and dtypes are checked here before the call
so that mistakes surface as Python exceptions.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree library; GWGEN_LIB names another build of it (the host-only
# sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("GWGEN_LIB") or os.path.join(_HERE, "libgwgen.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EHIP, GW_EUNSUPPORTED = 0, -1, -2, -3, -4
STATUS_NONFINITE_PSD = 1
STATUS_NONPOSITIVE_PSD = 2
STATUS_NONFINITE_DATA = 4
STATUS_CUT_AT_NYQUIST = 8
STATUS_SURROGATE_FALLBACK = 16
SCRATCH_BYTES = 64 << 20   # GW_SCRATCH_BYTES
N_PARAMS = 12
(Q_N, Q_F, Q_P, Q_L, Q_K, Q_FW, Q_NDET, Q_NPARAMS) = range(8)

# names declared in include/gwgen.h
EXPORTS = ("gw_create", "gw_destroy", "gw_strerror", "gw_last_error", "gw_query",
           "gw_workspace_size", "sample_params", "gen_fd_waveform", "project_detectors",
           "inject", "welch_psd", "whiten", "gw_generate_batch",
           "gw_surrogate_create", "gw_surrogate_destroy", "gw_surrogate_last_error",
           "gw_surrogate_n_weights", "gw_surrogate_set_weights", "gw_surrogate_get_weights",
           "gw_surrogate_targets", "gw_surrogate_fit_basis", "gw_surrogate_project",
           "gw_surrogate_fit_skip", "gw_surrogate_standardise", "gw_surrogate_forward",
           "gw_surrogate_gradients", "gw_surrogate_train_step", "gw_surrogate_hidden",
           "gw_surrogate_set_head", "gw_surrogate_fit_head", "gw_surrogate_nodes",
           "gw_surrogate_waveform", "gw_mismatch", "gw_mismatch_max", "gw_surrogate_save", "gw_surrogate_load",
           "gw_surrogate_set_state", "gw_workspace_size_surrogate", "gw_generate_batch_surrogate",
           "gw_graph_create", "gw_graph_launch", "gw_graph_set_batch", "gw_graph_last_error",
           "gw_graph_destroy", "gw_set_tuning", "gw_get_tuning", "gw_autotune",
           "gw_ragged_create", "gw_ragged_destroy", "gw_ragged_last_error", "gw_ragged_query",
           "gw_ragged_offsets", "gw_generate_ragged", "gw_ragged_graph_create",
           "gw_ragged_set_tuning", "gw_ragged_get_tuning", "gw_ragged_autotune",
           "gw_run_psd_workspace_size", "gw_run_psd", "gw_whiten_filter", "gw_generate_batch_runpsd",
           "gw_generate_batch_pairs", "gw_generate_batch_oversampled", "gw_surrogate_set_adam",
           "gw_surrogate_get_state", "gw_generate_batch_noalloc")

TUNE_ORD_WINDOW, TUNE_ORD_WELCH, TUNE_OCC_WELCH = 1, 2, 3
RTUNE_ORD_WINDOW, RTUNE_ORD_WELCH, RTUNE_GRID_WINDOW, RTUNE_GRID_WELCH, RTUNE_WINDOW_MODE = 1, 2, 3, 4, 5
RTUNE_WELCH_MODE = 6
(RQ_B, RQ_OUT_FLOATS, RQ_PSD_FLOATS, RQ_WORKSPACE, RQ_PSD_OFFSET, RQ_NCLASSES) = range(6)
RAGGED_MAX_CLASSES = 8


class GWConfig(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("det_id", ctypes.c_int32 * 4),
                ("fs", ctypes.c_double), ("t_window", ctypes.c_double),
                ("psd_length", ctypes.c_double), ("fftlen", ctypes.c_double),
                ("overlap", ctypes.c_double), ("f_min", ctypes.c_double),
                ("approximant", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mc", ctypes.c_double * 2), ("q", ctypes.c_double * 2),
                ("chi", ctypes.c_double * 2), ("dl", ctypes.c_double * 2),
                ("f0", ctypes.c_double * 2), ("quality", ctypes.c_double * 2),
                ("hrss", ctypes.c_double * 2)]


_LIB = None


def lib():
    """Load the in-tree library; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgwgen.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2407_19048_amd.build); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32
        sig = {
            "gw_create": ([ctypes.POINTER(GWConfig), ctypes.POINTER(vp)], i32),
            "gw_destroy": ([vp], i32),
            "gw_strerror": ([i32], ctypes.c_char_p),
            "gw_last_error": ([vp], ctypes.c_char_p),
            "gw_query": ([vp, i32, ctypes.POINTER(i64)], i32),
            "gw_workspace_size": ([vp, i64, ctypes.POINTER(i64)], i32),
            "sample_params": ([vp, u64, u64, i64, i64, vp, vp, vp], i32),
            "gen_fd_waveform": ([vp, vp, i64, vp, vp, vp], i32),
            "project_detectors": ([vp, vp, vp, vp, i64, vp, vp], i32),
            "inject": ([vp, vp, i64, vp, vp, i64, vp, vp], i32),
            "welch_psd": ([vp, vp, i64, vp, i64, vp, vp], i32),
            "whiten": ([vp, vp, vp, i64, vp, vp, vp], i32),
            "gw_generate_batch": ([vp, u64, u64, i64, vp, i64, vp, vp, vp, vp, i64, vp], i32),
            "gw_generate_batch_noalloc": ([vp, u64, u64, i64, vp, i64, vp, vp, vp, vp], i32),
            "gw_surrogate_create": ([vp, i64, ctypes.POINTER(vp)], i32),
            "gw_surrogate_destroy": ([vp], i32),
            "gw_surrogate_last_error": ([vp], ctypes.c_char_p),
            "gw_surrogate_n_weights": ([], i64),
            "gw_surrogate_set_weights": ([vp, vp, i64], i32),
            "gw_surrogate_get_weights": ([vp, vp, i64], i32),
            "gw_surrogate_targets": ([vp, vp, i64, vp, vp, vp, vp], i32),
            "gw_surrogate_fit_basis": ([vp, vp, vp, i64, vp], i32),
            "gw_surrogate_project": ([vp, vp, vp, i64, vp, vp], i32),
            "gw_surrogate_fit_skip": ([vp, vp, vp, i64, vp, vp], i32),
            "gw_surrogate_standardise": ([vp, vp, vp, i64, vp, vp], i32),
            "gw_surrogate_forward": ([vp, vp, i64, vp, vp], i32),
            "gw_surrogate_gradients": ([vp, vp, vp, i64, vp, vp, vp], i32),
            "gw_surrogate_train_step": ([vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, vp, vp], i32),
            "gw_surrogate_hidden": ([vp, vp, i64, vp, vp], i32),
            "gw_surrogate_set_head": ([vp, vp, i64], i32),
            "gw_surrogate_fit_head": ([vp, vp, vp, i64, ctypes.c_double], i32),
            "gw_surrogate_nodes": ([vp, vp, i64, vp, vp, vp], i32),
            "gw_surrogate_waveform": ([vp, vp, vp, i64, vp, vp, vp], i32),
            "gw_mismatch": ([vp, vp, vp, vp, vp, i64, vp, vp], i32),
            "gw_mismatch_max": ([vp, vp, vp, vp, vp, i64, vp, vp], i32),
            "gw_surrogate_save": ([vp, ctypes.c_char_p], i32),
            "gw_surrogate_load": ([vp, ctypes.c_char_p], i32),
            "gw_surrogate_set_state": ([vp, vp, vp, vp, vp, vp, vp], i32),
            "gw_surrogate_get_state": ([vp, vp, vp, vp, vp, vp, vp], i32),
            "gw_surrogate_set_adam": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double], i32),
            "gw_workspace_size_surrogate": ([vp, i64, ctypes.POINTER(i64)], i32),
            "gw_generate_batch_surrogate": ([vp, vp, u64, u64, i64, vp, i64, vp, vp, vp, ctypes.c_float, vp,
                                             i64, vp], i32),
            "gw_graph_create": ([vp, u64, u64, i64, vp, i64, vp, vp, vp, vp, i64, ctypes.POINTER(vp)], i32),
            "gw_graph_launch": ([vp, vp], i32),
            "gw_graph_set_batch": ([vp, u64, vp], i32),
            "gw_graph_last_error": ([vp], ctypes.c_char_p),
            "gw_graph_destroy": ([vp], i32),
            "gw_set_tuning": ([vp, i32, i64], i32),
            "gw_get_tuning": ([vp, i32, ctypes.POINTER(i64)], i32),
            "gw_autotune": ([vp, i64, vp, i64, vp, vp, i64, i32, vp], i32),
            "gw_ragged_create": ([ctypes.POINTER(GWConfig), i32, vp, i64, ctypes.POINTER(vp)], i32),
            "gw_ragged_destroy": ([vp], i32),
            "gw_ragged_last_error": ([vp], ctypes.c_char_p),
            "gw_ragged_query": ([vp, i32, ctypes.POINTER(i64)], i32),
            "gw_ragged_offsets": ([vp, vp, vp], i32),
            "gw_generate_ragged": ([vp, u64, u64, vp, vp, vp, vp, vp, vp, i64, vp], i32),
            "gw_ragged_graph_create": ([vp, u64, u64, vp, vp, vp, vp, vp, vp, i64, ctypes.POINTER(vp)], i32),
            "gw_ragged_set_tuning": ([vp, i32, i64], i32),
            "gw_ragged_get_tuning": ([vp, i32, ctypes.POINTER(i64)], i32),
            "gw_ragged_autotune": ([vp, vp, vp, vp, vp, i64, i32, vp], i32),
            "gw_run_psd_workspace_size": ([vp, i64, ctypes.POINTER(i64)], i32),
            "gw_run_psd": ([vp, vp, i64, i64, vp, vp, i64, vp], i32),
            "gw_whiten_filter": ([vp, vp, i64, vp, vp, vp], i32),
            "gw_generate_batch_runpsd": ([vp, u64, u64, i64, vp, i64, vp, i64, vp, vp, vp, vp, i64, vp], i32),
            "gw_generate_batch_pairs": ([vp, u64, u64, i64, vp, i64, vp, vp, vp, vp, vp, i64, vp], i32),
            "gw_generate_batch_oversampled": ([vp, u64, u64, i64, i32, vp, i64, vp, vp, vp, vp, i64, vp], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def make_config(cfg):
    """gw_config from a configuration dict (see inputs.CONFIGS)."""
    c = GWConfig()
    ids = list(cfg["det_ids"])
    c.n_det = len(ids)
    for i in range(4):
        c.det_id[i] = ids[i] if i < len(ids) else 0
    c.fs, c.t_window = float(cfg["fs"]), float(cfg["t_window"])
    c.psd_length, c.fftlen = float(cfg["psd_length"]), float(cfg["fftlen"])
    c.overlap, c.f_min = float(cfg["overlap"]), float(cfg["f_min"])
    c.approximant, c.precision = int(cfg["approximant"]), int(cfg.get("precision", 1))
    for name in ("mc", "q", "chi", "dl"):
        arr = getattr(c, name)
        arr[0], arr[1] = float(cfg[name][0]), float(cfg[name][1])
    for name in ("f0", "quality", "hrss"):
        arr = getattr(c, name)
        lo, hi = cfg.get(name, (0.0, 0.0))
        arr[0], arr[1] = float(lo), float(hi)
    return c


class GWError(RuntimeError):
    pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace_bytes(workspace):
    """Size in bytes of a workspace tensor, which must be contiguous device memory."""
    if workspace.device.type != "cuda" or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    return workspace.numel() * workspace.element_size()


def _want(t, dtype, shape, name):
    import torch
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class Generator:
    """One gw_ctx on the current device."""

    def __init__(self, cfg):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        h = ctypes.c_void_p()
        s = lib().gw_create(ctypes.byref(self._c), ctypes.byref(h))
        if s != GW_OK:
            raise GWError("gw_create failed: %s" % lib().gw_strerror(s).decode())
        self._h = h
        q = {}
        for key, name in ((Q_N, "N"), (Q_F, "F"), (Q_P, "P"), (Q_L, "L"), (Q_K, "K"),
                          (Q_FW, "Fw"), (Q_NDET, "D")):
            v = ctypes.c_int64()
            lib().gw_query(self._h, key, ctypes.byref(v))
            q[name] = v.value
        self.sizes = q

    def close(self):
        if getattr(self, "_h", None):
            lib().gw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s, what):
        if s != GW_OK:
            msg = lib().gw_last_error(self._h).decode()
            raise GWError("%s: %s (%s)" % (what, lib().gw_strerror(s).decode(), msg))

    def workspace_size(self, B):
        v = ctypes.c_int64()
        self._check(lib().gw_workspace_size(self._h, int(B), ctypes.byref(v)), "gw_workspace_size")
        return v.value

    # -- the six steps ---------------------------------------------------
    def sample_params(self, seed, first_index, B, L_bg, params, offset):
        import torch
        _want(params, torch.float64, (N_PARAMS, B), "params")
        _want(offset, torch.int64, (B,), "offset")
        self._check(lib().sample_params(self._h, int(seed), int(first_index), int(B), int(L_bg),
                                        _ptr(params), _ptr(offset), _stream()), "sample_params")

    def gen_fd_waveform(self, params, hp, hc):
        import torch
        B = params.shape[1]
        _want(params, torch.float64, (N_PARAMS, B), "params")
        _want(hp, torch.complex64, (B, self.sizes["F"]), "hp")
        _want(hc, torch.complex64, (B, self.sizes["F"]), "hc")
        self._check(lib().gen_fd_waveform(self._h, _ptr(params), B, _ptr(hp), _ptr(hc), _stream()),
                    "gen_fd_waveform")

    def project_detectors(self, params, hp, hc, hdet):
        import torch
        B = params.shape[1]
        _want(params, torch.float64, (N_PARAMS, B), "params")
        _want(hdet, torch.complex64, (B, self.sizes["D"], self.sizes["F"]), "hdet")
        _want(hp, torch.complex64, (B, self.sizes["F"]), "hp")
        _want(hc, torch.complex64, (B, self.sizes["F"]), "hc")
        self._check(lib().project_detectors(self._h, _ptr(params), _ptr(hp), _ptr(hc), B, _ptr(hdet),
                                            _stream()), "project_detectors")

    def inject(self, bg, offset, hdet, strain):
        import torch
        B = offset.shape[0]
        _want(offset, torch.int64, (B,), "offset")
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(hdet, torch.complex64, (B, self.sizes["D"], self.sizes["F"]), "hdet")
        _want(strain, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "strain")
        self._check(lib().inject(self._h, _ptr(bg), bg.shape[1], _ptr(offset), _ptr(hdet), B,
                                 _ptr(strain), _stream()), "inject")

    def welch_psd(self, bg, offset, psd):
        import torch
        B = offset.shape[0]
        _want(offset, torch.int64, (B,), "offset")
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(psd, torch.float32, (B, self.sizes["D"], self.sizes["Fw"]), "psd")
        self._check(lib().welch_psd(self._h, _ptr(bg), bg.shape[1], _ptr(offset), B, _ptr(psd),
                                    _stream()), "welch_psd")

    def whiten(self, strain, psd, out, status=None):
        import torch
        B = strain.shape[0]
        _want(strain, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "strain")
        _want(psd, torch.float32, (B, self.sizes["D"], self.sizes["Fw"]), "psd")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        self._check(lib().whiten(self._h, _ptr(strain), _ptr(psd), B, _ptr(out), _ptr(status),
                                 _stream()), "whiten")

    def generate_batch(self, seed, batch_index, B, bg, out, workspace, params_f32=None, status=None):
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_generate_batch(self._h, int(seed), int(batch_index), int(B), _ptr(bg),
                                            bg.shape[1], _ptr(out), _ptr(params_f32), _ptr(status),
                                            _ptr(workspace), nbytes, _stream()),
                    "gw_generate_batch")

    def generate_batch_noalloc(self, seed, batch_index, B, bg, out, params_f32=None, status=None):
        """gw_generate_batch on the library's static scratch area (no workspace)."""
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        self._check(lib().gw_generate_batch_noalloc(self._h, int(seed), int(batch_index), int(B), _ptr(bg),
                                                    bg.shape[1], _ptr(out), _ptr(params_f32), _ptr(status),
                                                    _stream()), "gw_generate_batch_noalloc")

    def mismatch(self, ha, hb, psd, params, mm):
        """Noise-weighted mismatch per sample (see gw_mismatch)."""
        import torch
        B = ha.shape[0]
        _want(ha, torch.complex64, (B, self.sizes["F"]), "ha")
        _want(hb, torch.complex64, (B, self.sizes["F"]), "hb")
        _want(psd, torch.float32, (self.sizes["F"],), "psd")
        _want(mm, torch.float64, (B,), "mm")
        if params is not None:
            _want(params, torch.float64, (N_PARAMS, B), "params")
        self._check(lib().gw_mismatch(self._h, _ptr(ha), _ptr(hb), _ptr(psd), _ptr(params), B, _ptr(mm),
                                      _stream()), "gw_mismatch")

    def mismatch_max(self, ha, hb, psd, params, mm):
        """Mismatch maximised over a time and a phase shift (see gw_mismatch_max)."""
        import torch
        B = ha.shape[0]
        _want(ha, torch.complex64, (B, self.sizes["F"]), "ha")
        _want(hb, torch.complex64, (B, self.sizes["F"]), "hb")
        _want(psd, torch.float32, (self.sizes["F"],), "psd")
        _want(mm, torch.float64, (B,), "mm")
        if params is not None:
            _want(params, torch.float64, (N_PARAMS, B), "params")
        self._check(lib().gw_mismatch_max(self._h, _ptr(ha), _ptr(hb), _ptr(psd), _ptr(params), B, _ptr(mm),
                                          _stream()), "gw_mismatch_max")

    def alloc_workspace_surrogate(self, B, device="cuda"):
        import torch
        v = ctypes.c_int64()
        self._check(lib().gw_workspace_size_surrogate(self._h, int(B), ctypes.byref(v)),
                    "gw_workspace_size_surrogate")
        return torch.empty((v.value + 7) // 8, dtype=torch.float64, device=device)

    def generate_batch_surrogate(self, surrogate, seed, batch_index, B, bg, out, workspace, params_f32=None,
                                 status=None, log10_mm_max=-3.0):
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_generate_batch_surrogate(self._h, surrogate._h, int(seed), int(batch_index), int(B),
                                                      _ptr(bg), bg.shape[1], _ptr(out), _ptr(params_f32),
                                                      _ptr(status), ctypes.c_float(log10_mm_max),
                                                      _ptr(workspace), nbytes, _stream()),
                    "gw_generate_batch_surrogate")

    def workspace_views(self, workspace, B):
        """(params float64 [12][B], offsets int64 [B]) inside a batch workspace."""
        import torch
        pb = ((B * 12 * 8 + 255) // 256) * 256
        raw = workspace.view(torch.uint8)
        params = raw[:B * 12 * 8].view(torch.float64).view(N_PARAMS, B)
        offs = raw[pb:pb + B * 8].view(torch.int64)
        return params, offs

    def alloc_workspace(self, B, device="cuda"):
        import torch
        n = self.workspace_size(B)
        return torch.empty((n + 7) // 8, dtype=torch.float64, device=device)

    # -- view pairs and oversampling ---------------------------------------
    def generate_batch_pairs(self, seed, batch_index, B, bg, out_ref, out_shift, workspace, params_f32=None,
                             status=None):
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        for t, nm in ((out_ref, "out_ref"), (out_shift, "out_shift")):
            _want(t, torch.float32, (B, self.sizes["D"], self.sizes["N"]), nm)
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_generate_batch_pairs(self._h, int(seed), int(batch_index), int(B), _ptr(bg),
                                                  bg.shape[1], _ptr(out_ref), _ptr(out_shift), _ptr(params_f32),
                                                  _ptr(status), _ptr(workspace), nbytes, _stream()),
                    "gw_generate_batch_pairs")

    def generate_batch_oversampled(self, seed, batch_index, B, ext_k, bg, out, workspace, params_f32=None,
                                   status=None):
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_generate_batch_oversampled(self._h, int(seed), int(batch_index), int(B), int(ext_k),
                                                        _ptr(bg), bg.shape[1], _ptr(out), _ptr(params_f32),
                                                        _ptr(status), _ptr(workspace), nbytes, _stream()),
                    "gw_generate_batch_oversampled")

    # -- per-run PSD mode -------------------------------------------------
    def run_psd(self, bg, n_chunks, psd):
        """Per-detector Welch PSD over the first n_chunks*K segments of bg."""
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(psd, torch.float32, (self.sizes["D"], self.sizes["Fw"]), "psd")
        v = ctypes.c_int64()
        self._check(lib().gw_run_psd_workspace_size(self._h, int(n_chunks), ctypes.byref(v)),
                    "gw_run_psd_workspace_size")
        ws = torch.empty((v.value + 7) // 8, dtype=torch.float64, device=bg.device)
        self._check(lib().gw_run_psd(self._h, _ptr(bg), bg.shape[1], int(n_chunks), _ptr(psd), _ptr(ws),
                                     v.value, _stream()), "gw_run_psd")
        return ws  # keep alive until the stream has run

    def whiten_filter(self, psd, M, filt, status=None):
        import torch
        _want(psd, torch.float32, (self.sizes["D"], self.sizes["Fw"]), "psd")
        _want(filt, torch.float32, (self.sizes["D"], self.sizes["F"]), "filt")
        if status is not None:
            _want(status, torch.int32, (self.sizes["D"],), "status")
        self._check(lib().gw_whiten_filter(self._h, _ptr(psd), int(M), _ptr(filt), _ptr(status), _stream()),
                    "gw_whiten_filter")

    def generate_batch_runpsd(self, seed, batch_index, B, bg, filt, crop, out, workspace, params_f32=None,
                              status=None):
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(filt, torch.float32, (self.sizes["D"], self.sizes["F"]), "filt")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"] - 2 * int(crop)), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_generate_batch_runpsd(self._h, int(seed), int(batch_index), int(B), _ptr(bg),
                                                   bg.shape[1], _ptr(filt), int(crop), _ptr(out),
                                                   _ptr(params_f32), _ptr(status), _ptr(workspace), nbytes,
                                                   _stream()), "gw_generate_batch_runpsd")

    # -- graphs and tuning ------------------------------------------------
    def graph(self, seed, first_batch, B, bg, out, workspace, params_f32=None, status=None):
        """Captured gw_generate_batch; each launch advances the batch index."""
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (B,), "status")
        h = ctypes.c_void_p()
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_graph_create(self._h, int(seed), int(first_batch), int(B), _ptr(bg), bg.shape[1],
                                          _ptr(out), _ptr(params_f32), _ptr(status), _ptr(workspace), nbytes,
                                          ctypes.byref(h)), "gw_graph_create")
        return Graph(h, keep=(bg, out, workspace, params_f32, status))

    def set_tuning(self, key, value):
        self._check(lib().gw_set_tuning(self._h, int(key), int(value)), "gw_set_tuning")

    def get_tuning(self, key):
        v = ctypes.c_int64()
        self._check(lib().gw_get_tuning(self._h, int(key), ctypes.byref(v)), "gw_get_tuning")
        return v.value

    def autotune(self, B, bg, out, workspace, reps=5):
        """Pick the radix orders; returns the mean ms per variant."""
        import torch
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(out, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "out")
        rep = (ctypes.c_double * 6)()
        nbytes = _workspace_bytes(workspace)
        self._check(lib().gw_autotune(self._h, int(B), _ptr(bg), bg.shape[1], _ptr(out), _ptr(workspace), nbytes,
                                      int(reps), ctypes.cast(rep, ctypes.c_void_p)), "gw_autotune")
        return {"welch_ord0_occ2": rep[0], "welch_ord1_occ2": rep[1], "welch_ord0_occ3": rep[2],
                "welch_ord1_occ3": rep[3], "window_ord0": rep[4], "window_ord1": rep[5]}


class Graph:
    """A captured batch pipeline (gw_graph)."""

    def __init__(self, h, keep):
        self._h = h
        self._keep = keep  # the buffers the graph was captured with

    def launch(self):
        s = lib().gw_graph_launch(self._h, _stream())
        if s != GW_OK:
            raise GWError("gw_graph_launch: %s" % lib().gw_graph_last_error(self._h).decode())

    def set_batch(self, batch_index):
        s = lib().gw_graph_set_batch(self._h, int(batch_index), _stream())
        if s != GW_OK:
            raise GWError("gw_graph_set_batch: %s" % lib().gw_graph_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().gw_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ragged:
    """A gw_ragged plan: B signal slots, each of one size class."""

    def __init__(self, classes, cls):
        import numpy as np
        self.classes = [dict(c) for c in classes]
        n = len(self.classes)
        if not 1 <= n <= RAGGED_MAX_CLASSES:
            raise ValueError("1..%d classes" % RAGGED_MAX_CLASSES)
        self.cls = np.ascontiguousarray(cls, dtype=np.int32)
        self.B = int(self.cls.shape[0])
        arr = (GWConfig * n)(*[make_config(c) for c in self.classes])
        self._cfgs = arr
        h = ctypes.c_void_p()
        s = lib().gw_ragged_create(arr, n, self.cls.ctypes.data_as(ctypes.c_void_p), self.B, ctypes.byref(h))
        if s != GW_OK:
            raise GWError("gw_ragged_create failed: %s" % lib().gw_strerror(s).decode())
        self._h = h
        self.D = len(self.classes[0]["det_ids"])
        self.out_floats = self._query(RQ_OUT_FLOATS)
        self.psd_floats = self._query(RQ_PSD_FLOATS)
        self.workspace_bytes = self._query(RQ_WORKSPACE)
        self.psd_byte_offset = self._query(RQ_PSD_OFFSET)
        self.out_offset = np.zeros(self.B + 1, dtype=np.int64)
        self.psd_offset = np.zeros(self.B + 1, dtype=np.int64)
        s = lib().gw_ragged_offsets(self._h, self.out_offset.ctypes.data_as(ctypes.c_void_p),
                                    self.psd_offset.ctypes.data_as(ctypes.c_void_p))
        self._check(s, "gw_ragged_offsets")

    def _check(self, s, what):
        if s != GW_OK:
            msg = lib().gw_ragged_last_error(self._h).decode()
            raise GWError("%s: %s (%s)" % (what, lib().gw_strerror(s).decode(), msg))

    def _query(self, key):
        v = ctypes.c_int64()
        self._check(lib().gw_ragged_query(self._h, key, ctypes.byref(v)), "gw_ragged_query")
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            lib().gw_ragged_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_workspace(self, device="cuda"):
        import torch
        return torch.empty((self.workspace_bytes + 7) // 8, dtype=torch.float64, device=device)

    def alloc_out(self, device="cuda"):
        import torch
        return torch.empty(self.out_floats, dtype=torch.float32, device=device)

    def _bg_arrays(self, bgs):
        """bgs: list (one per class) of float32 device tensors [D][L_bg]."""
        import torch
        if len(bgs) != len(self.classes):
            raise ValueError("one background per class")
        for b in bgs:
            _want(b, torch.float32, (self.D, b.shape[1]), "bg")
        n = len(bgs)
        ptrs = (ctypes.c_void_p * n)(*[b.data_ptr() for b in bgs])
        lens = (ctypes.c_int64 * n)(*[b.shape[1] for b in bgs])
        return ptrs, lens

    def _common(self, out, workspace, params_f32, status):
        import torch
        _want(out, torch.float32, (self.out_floats,), "out")
        if params_f32 is not None:
            _want(params_f32, torch.float32, (N_PARAMS, self.B), "params_f32")
        if status is not None:
            _want(status, torch.int32, (self.B,), "status")
        return _workspace_bytes(workspace)

    def generate(self, seed, batch_index, bgs, out, workspace, params_f32=None, status=None):
        nbytes = self._common(out, workspace, params_f32, status)
        ptrs, lens = self._bg_arrays(bgs)
        self._check(lib().gw_generate_ragged(self._h, int(seed), int(batch_index), ctypes.cast(ptrs, ctypes.c_void_p),
                                             ctypes.cast(lens, ctypes.c_void_p), _ptr(out), _ptr(params_f32),
                                             _ptr(status), _ptr(workspace), nbytes, _stream()),
                    "gw_generate_ragged")

    def graph(self, seed, first_batch, bgs, out, workspace, params_f32=None, status=None):
        nbytes = self._common(out, workspace, params_f32, status)
        ptrs, lens = self._bg_arrays(bgs)
        h = ctypes.c_void_p()
        self._check(lib().gw_ragged_graph_create(self._h, int(seed), int(first_batch),
                                                 ctypes.cast(ptrs, ctypes.c_void_p),
                                                 ctypes.cast(lens, ctypes.c_void_p), _ptr(out), _ptr(params_f32),
                                                 _ptr(status), _ptr(workspace), nbytes, ctypes.byref(h)),
                    "gw_ragged_graph_create")
        return Graph(h, keep=(tuple(bgs), out, workspace, params_f32, status))

    def set_tuning(self, key, value):
        self._check(lib().gw_ragged_set_tuning(self._h, int(key), int(value)), "gw_ragged_set_tuning")

    def get_tuning(self, key):
        v = ctypes.c_int64()
        self._check(lib().gw_ragged_get_tuning(self._h, int(key), ctypes.byref(v)), "gw_ragged_get_tuning")
        return v.value

    def autotune(self, bgs, out, workspace, reps=3):
        """Pick radix orders, the Welch issue mode and grid; returns the timing table [ms]."""
        nbytes = self._common(out, workspace, None, None)
        ptrs, lens = self._bg_arrays(bgs)
        rep = (ctypes.c_double * 12)()
        self._check(lib().gw_ragged_autotune(self._h, ctypes.cast(ptrs, ctypes.c_void_p),
                                             ctypes.cast(lens, ctypes.c_void_p), _ptr(out), _ptr(workspace),
                                             nbytes, int(reps), ctypes.cast(rep, ctypes.c_void_p)),
                    "gw_ragged_autotune")
        return {"welch": {(o, g): rep[o * 3 + i] for o in (0, 1) for i, g in enumerate((1, 2, 4))},
                "window": {(m, o): rep[6 + 2 * m + o] for m in (0, 1) for o in (0, 1)},
                "welch_class": {o: rep[10 + o] for o in (0, 1)}}

    def signal(self, out, i):
        """View [D][N_i] of signal slot i in the flat output."""
        a, b = int(self.out_offset[i]), int(self.out_offset[i + 1])
        return out[a:b].view(self.D, (b - a) // self.D)

    def workspace_views(self, workspace):
        """(params float64 [12][B], offsets int64 [B], flat PSD float32) in the workspace."""
        import torch
        B = self.B
        pb = ((B * 12 * 8 + 255) // 256) * 256
        raw = workspace.view(torch.uint8)
        params = raw[:B * 12 * 8].view(torch.float64).view(N_PARAMS, B)
        offs = raw[pb:pb + B * 8].view(torch.int64)
        psd = raw[self.psd_byte_offset:self.psd_byte_offset + 4 * self.psd_floats].view(torch.float32)
        return params, offs, psd
