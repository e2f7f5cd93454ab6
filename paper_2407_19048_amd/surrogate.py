"""Learned waveform surrogate: ctypes wrapper of the gw_surrogate_* entry
points and the training driver.

The training loop only sequences C-ABI calls: prior draws and plain-model targets
on the GPU, basis fit, skip-path fit, AdamW steps of the bfloat16 MFMA
forward/backward kernels, and the fit of the mismatch head.  Weight
initialisation draws seeded random numbers on the host and hands them over.
"""

import ctypes
import math
import time

import numpy as np

from .gwgen import GWError, _ptr, _stream, _want, lib

NODES = 1024
N_OUT = 128
N_FEAT = 9
HIDDEN = 256
LAYERS = ((16, 256), (256, 256), (256, 256), (256, 128))


def init_weights(seed, scale=1.0):
    """He-style initial weights in the flat layout (input rows 4..15 zero)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l, (nin, nout) in enumerate(LAYERS):
        fan_in = 4 if l == 0 else nin
        W = rng.standard_normal((nin, nout)) * scale * math.sqrt(2.0 / fan_in)
        if l == 0:
            W[4:] = 0.0
        if l == len(LAYERS) - 1:
            W *= 0.1
        parts += [W.astype(np.float32).ravel(), np.zeros(nout, np.float32)]
    return np.concatenate(parts)


class Surrogate:
    def __init__(self, gen, max_batch=8192):
        self.gen = gen
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        s = lib().gw_surrogate_create(gen._h, self.max_batch, ctypes.byref(h))
        if s != 0:
            raise GWError("gw_surrogate_create failed (%d): %s" % (s, lib().gw_last_error(gen._h).decode()))
        self._h = h
        self.n_weights = lib().gw_surrogate_n_weights()
        self.history = []

    def close(self):
        if getattr(self, "_h", None):
            lib().gw_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s, what):
        if s != 0:
            raise GWError("%s failed (%d): %s" % (what, s, lib().gw_surrogate_last_error(self._h).decode()))

    # ----------------------------------------------------------- weights
    def set_weights(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(lib().gw_surrogate_set_weights(self._h, flat.ctypes.data, flat.size), "set_weights")

    def get_weights(self):
        out = np.empty(self.n_weights, dtype=np.float32)
        self._check(lib().gw_surrogate_get_weights(self._h, out.ctypes.data, out.size), "get_weights")
        return out

    def set_head(self, head):
        head = np.ascontiguousarray(head, dtype=np.float32)
        self._check(lib().gw_surrogate_set_head(self._h, head.ctypes.data, head.size), "set_head")

    def set_state(self, basis, mean, A, zmean, zstd, head):
        """Non-network state from host arrays (see gw_surrogate_set_state)."""
        arrs = [np.ascontiguousarray(basis, np.float32), np.ascontiguousarray(mean, np.float64),
                np.ascontiguousarray(A, np.float32), np.ascontiguousarray(zmean, np.float32),
                np.ascontiguousarray(zstd, np.float32), np.ascontiguousarray(head, np.float32)]
        shapes = [(2, 64, NODES), (2, NODES), (N_FEAT, N_OUT), (N_OUT,), (N_OUT,), (HIDDEN + 1,)]
        for a, sh in zip(arrs, shapes):
            if a.shape != sh:
                raise ValueError("state array shape %s, expected %s" % (a.shape, sh))
        self._check(lib().gw_surrogate_set_state(self._h, *[a.ctypes.data for a in arrs]), "set_state")

    def get_state(self):
        """(basis, mean, A, zmean, zstd, head) as host arrays."""
        arrs = [np.empty((2, 64, NODES), np.float32), np.empty((2, NODES), np.float64),
                np.empty((N_FEAT, N_OUT), np.float32), np.empty(N_OUT, np.float32), np.empty(N_OUT, np.float32),
                np.empty(HIDDEN + 1, np.float32)]
        self._check(lib().gw_surrogate_get_state(self._h, *[a.ctypes.data for a in arrs]), "get_state")
        return tuple(arrs)

    def set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(lib().gw_surrogate_set_adam(self._h, ctypes.c_double(beta1), ctypes.c_double(beta2),
                                                ctypes.c_double(eps)), "set_adam")

    def save(self, path):
        self._check(lib().gw_surrogate_save(self._h, path.encode()), "save")

    def load(self, path):
        self._check(lib().gw_surrogate_load(self._h, path.encode()), "load")

    # ------------------------------------------------------------- pieces
    def targets(self, params, ratio, dpsi, feat):
        B = params.shape[1]
        self._check(lib().gw_surrogate_targets(self._h, _ptr(params), B, _ptr(ratio), _ptr(dpsi), _ptr(feat),
                                               _stream()), "targets")

    def fit_basis(self, ratio, dpsi):
        self._check(lib().gw_surrogate_fit_basis(self._h, _ptr(ratio), _ptr(dpsi), ratio.shape[0], _stream()),
                    "fit_basis")

    def project(self, ratio, dpsi, C):
        self._check(lib().gw_surrogate_project(self._h, _ptr(ratio), _ptr(dpsi), ratio.shape[0], _ptr(C),
                                               _stream()), "project")

    def fit_skip(self, feat, C, Z):
        self._check(lib().gw_surrogate_fit_skip(self._h, _ptr(feat), _ptr(C), C.shape[0], _ptr(Z), _stream()),
                    "fit_skip")

    def forward(self, theta, out):
        self._check(lib().gw_surrogate_forward(self._h, _ptr(theta), theta.shape[0], _ptr(out), _stream()),
                    "forward")

    def gradients(self, theta, z, grads, loss=None):
        self._check(lib().gw_surrogate_gradients(self._h, _ptr(theta), _ptr(z), theta.shape[0], _ptr(grads),
                                                 _ptr(loss), _stream()), "gradients")

    def train_step(self, theta, z, lr, weight_decay=0.0, loss=None):
        self._check(lib().gw_surrogate_train_step(self._h, _ptr(theta), _ptr(z), theta.shape[0],
                                                  ctypes.c_float(lr), ctypes.c_float(weight_decay),
                                                  _ptr(loss), _stream()), "train_step")

    def hidden(self, theta, h3):
        self._check(lib().gw_surrogate_hidden(self._h, _ptr(theta), theta.shape[0], _ptr(h3), _stream()),
                    "hidden")

    def nodes(self, params, nodes, logmm=None):
        B = params.shape[1]
        self._check(lib().gw_surrogate_nodes(self._h, _ptr(params), B, _ptr(nodes), _ptr(logmm), _stream()),
                    "nodes")

    def waveform(self, params, nodes, hp, hc):
        B = params.shape[1]
        self._check(lib().gw_surrogate_waveform(self._h, _ptr(params), _ptr(nodes), B, _ptr(hp), _ptr(hc),
                                                _stream()), "waveform")

    # ------------------------------------------------------------ training
    def _draw(self, seed, first, n):
        import torch
        params = torch.empty((12, n), dtype=torch.float64, device="cuda")
        offs = torch.empty(n, dtype=torch.int64, device="cuda")
        need = self.gen.sizes["P"] + self.gen.sizes["N"]
        self.gen.sample_params(seed, first, n, need, params, offs)
        return params

    def fit(self, seed=3, n_basis=32768, n_train=1 << 20, epochs=20, batch=8192, lr=2e-3, lr_min=2e-5,
            weight_decay=2e-3, n_head=8192, psd=None, log=None, init_seed=17):
        """Build the basis and skip path, train the MLP and fit the head.
        AdamW with weight decay 2e-3 by default, the setting section 5.1 of
        the paper uses for its own network."""
        import torch
        t0 = time.perf_counter()
        dev = "cuda"
        chunk = 32768
        # 1. basis from n_basis draws
        p = self._draw(seed, 0, n_basis)
        ratio = torch.empty((n_basis, NODES), dtype=torch.float32, device=dev)
        dpsi = torch.empty_like(ratio)
        feat = torch.empty((n_basis, N_FEAT), dtype=torch.float64, device=dev)
        self.targets(p, ratio, dpsi, feat)
        self.fit_basis(ratio, dpsi)
        del ratio, dpsi, feat, p
        # 2. training set: coefficients and features, chunk by chunk
        theta = torch.empty((n_train, 4), dtype=torch.float32, device=dev)
        C = torch.empty((n_train, N_OUT), dtype=torch.float32, device=dev)
        F = torch.empty((n_train, N_FEAT), dtype=torch.float64, device=dev)
        r_buf = torch.empty((chunk, NODES), dtype=torch.float32, device=dev)
        d_buf = torch.empty_like(r_buf)
        for i0 in range(0, n_train, chunk):
            n = min(chunk, n_train - i0)
            p = self._draw(seed, n_basis + i0, n)
            self.targets(p, r_buf[:n], d_buf[:n], F[i0:i0 + n])
            self.project(r_buf[:n], d_buf[:n], C[i0:i0 + n])
            theta[i0:i0 + n] = p[:4].t().float()
        del r_buf, d_buf
        Z = torch.empty_like(C)
        self.fit_skip(F, C, Z)
        del C, F
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        # 3. AdamW on the standardised residual targets, cosine learning rate
        self.set_weights(init_weights(init_seed))
        steps_per_epoch = n_train // batch
        total = steps_per_epoch * epochs
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        # loss of the initial network on the first batch (gradients only, no update)
        grads = torch.empty(self.n_weights, dtype=torch.float32, device=dev)
        self.gradients(theta[:batch], Z[:batch], grads, loss)
        torch.cuda.synchronize()
        initial_mse = float(loss.item()) / (batch * N_OUT)
        del grads
        step = 0
        for ep in range(epochs):
            shift = (ep * 7919 * batch // 13) % n_train
            for j in range(steps_per_epoch):
                i0 = (shift + j * batch) % (n_train - batch + 1)
                a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / total))
                want = (j == steps_per_epoch - 1)
                self.train_step(theta[i0:i0 + batch], Z[i0:i0 + batch], a, weight_decay, loss if want else None)
                step += 1
            torch.cuda.synchronize()
            mse = float(loss.item()) / (batch * N_OUT)
            self.history.append(mse)
            if log:
                log("surrogate epoch %d/%d: mse %.3e (lr %.2e)" % (ep + 1, epochs, mse, a))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0 - t_data
        # 4. mismatch head on held-out draws
        head_stats = None
        if psd is not None and n_head > 0:
            head_stats = self.fit_mismatch_head(seed + 1, n_head, psd)
        return dict(seconds_data=t_data, seconds_train=t_train, steps=total, initial_mse=initial_mse,
                    final_mse=self.history[-1], weight_decay=weight_decay, head=head_stats)

    def mismatch_vs_plain(self, params, psd, maximised=False):
        """(mm float64 [B], predicted log10 mm float32 [B]) against the plain
        model; with maximised, the mismatch minimised over a time shift and a
        phase offset (gw_mismatch_max) is appended as a third tensor."""
        import torch
        B = params.shape[1]
        F = self.gen.sizes["F"]
        nodes = torch.empty((B, 2, NODES), dtype=torch.float32, device="cuda")
        logmm = torch.empty(B, dtype=torch.float32, device="cuda")
        self.nodes(params, nodes, logmm)
        hs = torch.empty((B, F), dtype=torch.complex64, device="cuda")
        hsx = torch.empty_like(hs)
        self.waveform(params, nodes, hs, hsx)
        hp = torch.empty_like(hs)
        hx = torch.empty_like(hs)
        self.gen.gen_fd_waveform(params, hp, hx)
        mm = torch.empty(B, dtype=torch.float64, device="cuda")
        self.gen.mismatch(hs, hp, psd, params, mm)
        if not maximised:
            return mm, logmm
        mm_max = torch.empty_like(mm)
        self.gen.mismatch_max(hs, hp, psd, params, mm_max)
        return mm, logmm, mm_max

    def fit_mismatch_head(self, seed, n, psd):
        import torch
        p = self._draw(seed, 1 << 40, n)
        mm, _ = self.mismatch_vs_plain(p, psd)
        theta = p[:4].t().float().contiguous()
        h3 = torch.empty((n, HIDDEN), dtype=torch.float32, device="cuda")
        for i0 in range(0, n, self.max_batch):
            m = min(self.max_batch, n - i0)
            self.hidden(theta[i0:i0 + m], h3[i0:i0 + m])
        self.fit_head(h3, mm.cpu().numpy(), 1e-4)
        mm = mm.cpu().numpy()
        return dict(n=n, median_mm=float(np.median(mm)), p90_mm=float(np.percentile(mm, 90)))

    def fit_head(self, h3, mm, ridge):
        """Ridge fit of the log10-mismatch head (see gw_surrogate_fit_head);
        h3 device float [n][256], mm host mismatches [n]."""
        import torch
        n = h3.shape[0]
        _want(h3, torch.float32, (n, HIDDEN), "h3")
        mm = np.ascontiguousarray(mm, dtype=np.float64)
        if mm.shape != (n,):
            raise ValueError("mm must have shape (%d,)" % n)
        torch.cuda.synchronize()
        self._check(lib().gw_surrogate_fit_head(self._h, _ptr(h3), mm.ctypes.data, n, ctypes.c_double(ridge)),
                    "fit_head")
