"""ctypes binding of libgwgen.so (C ABI in include/gwgen.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Arrays are PyTorch device tensors; the library sees raw device pointers and
the current HIP stream.  Shapes and dtypes are checked here before the call
so that mistakes surface as Python exceptions.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgwgen.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EHIP, GW_EUNSUPPORTED = 0, -1, -2, -3, -4
STATUS_NONFINITE_PSD = 1
STATUS_NONPOSITIVE_PSD = 2
STATUS_NONFINITE_DATA = 4
STATUS_CUT_AT_NYQUIST = 8
STATUS_SURROGATE_FALLBACK = 16
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
           "gw_surrogate_waveform", "gw_mismatch", "gw_surrogate_save", "gw_surrogate_load",
           "gw_surrogate_set_state", "gw_workspace_size_surrogate", "gw_generate_batch_surrogate")


class GWConfig(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("det_id", ctypes.c_int32 * 4),
                ("fs", ctypes.c_double), ("t_window", ctypes.c_double),
                ("psd_length", ctypes.c_double), ("fftlen", ctypes.c_double),
                ("overlap", ctypes.c_double), ("f_min", ctypes.c_double),
                ("approximant", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mc", ctypes.c_double * 2), ("q", ctypes.c_double * 2),
                ("chi", ctypes.c_double * 2), ("dl", ctypes.c_double * 2)]


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
            "gw_surrogate_save": ([vp, ctypes.c_char_p], i32),
            "gw_surrogate_load": ([vp, ctypes.c_char_p], i32),
            "gw_surrogate_set_state": ([vp, vp, vp, vp, vp, vp, vp], i32),
            "gw_workspace_size_surrogate": ([vp, i64, ctypes.POINTER(i64)], i32),
            "gw_generate_batch_surrogate": ([vp, vp, u64, u64, i64, vp, i64, vp, vp, vp, ctypes.c_float, vp,
                                             i64, vp], i32),
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
    return c


class GWError(RuntimeError):
    pass


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


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
        _want(hdet, torch.complex64, (B, self.sizes["D"], self.sizes["F"]), "hdet")
        _want(hp, torch.complex64, (B, self.sizes["F"]), "hp")
        _want(hc, torch.complex64, (B, self.sizes["F"]), "hc")
        self._check(lib().project_detectors(self._h, _ptr(params), _ptr(hp), _ptr(hc), B, _ptr(hdet),
                                            _stream()), "project_detectors")

    def inject(self, bg, offset, hdet, strain):
        import torch
        B = offset.shape[0]
        _want(bg, torch.float32, (self.sizes["D"], bg.shape[1]), "bg")
        _want(hdet, torch.complex64, (B, self.sizes["D"], self.sizes["F"]), "hdet")
        _want(strain, torch.float32, (B, self.sizes["D"], self.sizes["N"]), "strain")
        self._check(lib().inject(self._h, _ptr(bg), bg.shape[1], _ptr(offset), _ptr(hdet), B,
                                 _ptr(strain), _stream()), "inject")

    def welch_psd(self, bg, offset, psd):
        import torch
        B = offset.shape[0]
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
        if workspace.device.type != "cuda" or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous device tensor")
        nbytes = workspace.numel() * workspace.element_size()
        self._check(lib().gw_generate_batch(self._h, int(seed), int(batch_index), int(B), _ptr(bg),
                                            bg.shape[1], _ptr(out), _ptr(params_f32), _ptr(status),
                                            _ptr(workspace), nbytes, _stream()),
                    "gw_generate_batch")

    def mismatch(self, ha, hb, psd, params, mm):
        """Noise-weighted mismatch per sample (see gw_mismatch)."""
        import torch
        B = ha.shape[0]
        _want(ha, torch.complex64, (B, self.sizes["F"]), "ha")
        _want(hb, torch.complex64, (B, self.sizes["F"]), "hb")
        _want(psd, torch.float32, (self.sizes["F"],), "psd")
        _want(mm, torch.float64, (B,), "mm")
        self._check(lib().gw_mismatch(self._h, _ptr(ha), _ptr(hb), _ptr(psd), _ptr(params), B, _ptr(mm),
                                      _stream()), "gw_mismatch")

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
        nbytes = workspace.numel() * workspace.element_size()
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
