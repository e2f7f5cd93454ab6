"""Seeded synthetic inputs shared by the HIP path and its checker.

Nothing here belongs to the generator's own arithmetic: this module builds
the workload configurations and the stand-in for the detector strain that
the paper keeps resident on the accelerator (section 3.2: a long two-detector
background chunk at 2048 Hz copied to device memory once before training).
The real strain is not available, so the background is stationary Gaussian
noise coloured to an analytic advanced-LIGO-like design curve.

Background recipe (per detector row, independent seeds):
  * target one-sided PSD (strain scale 2**70 applied, so values fit binary32)
        S_t(f) = 2**140 * 1e-49 * [x^-4.14 - 5 x^-2
                 + 111 (1 - x^2 + x^4/2) / (1 + x^2/2)],  x = max(f,10 Hz)/215 Hz
    (the analytic zero-detuned high-power fit of Ajith 2011);
  * FIR h of M = 4 s * fs taps: frequency-sampled design sqrt(fs S_t / 2),
    zero phase, rolled by M/2 and Hann-tapered;
  * noise = circular convolution of unit white Gaussian noise (numpy PCG64)
    with h over the whole row, so the row is exactly stationary with
    one-sided PSD S_true(f) = (2/fs) |sum_n h[n] exp(-2 pi i f n / fs)|^2.
"""

import math
import os

import numpy as np

DET_NAMES = {0: "H1", 1: "L1", 2: "V1"}

# Workload configurations.  Prior ranges replace those of the paper's
# Table 1 where the workload names them.
CONFIGS = {
    # 64 signals, H1+L1, 1024 Hz, 4 s windows, TaylorF2, Welch 32 s / 2 s / 50 %
    "pr1_plain": dict(
        det_ids=(0, 1), fs=1024.0, t_window=4.0, psd_length=32.0, fftlen=2.0,
        overlap=1.0, f_min=30.0, approximant=0, precision=1,
        mc=(10.0, 60.0), q=(0.25, 1.0), chi=(-0.9, 0.9), dl=(100.0, 2000.0),
        batch=64, log2_bg=22),
    # paper scale: 2048 signals, H1+L1+V1, 2048 Hz, 8 s, IMR-form, Welch 64 s
    "paper_scale": dict(
        det_ids=(0, 1, 2), fs=2048.0, t_window=8.0, psd_length=64.0, fftlen=2.0,
        overlap=1.0, f_min=20.0, approximant=1, precision=1,
        mc=(10.0, 100.0), q=(0.125, 1.0), chi=(-0.99, 0.99), dl=(100.0, 3100.0),
        batch=2048, log2_bg=27),
}
# sine-Gaussian bursts at the paper-scale shape (f0, Q, hrss ranges: a
# reading; the paper only names the morphology)
CONFIGS["sine_gaussian"] = dict(CONFIGS["paper_scale"], approximant=2, f0=(32.0, 1000.0), quality=(3.0, 30.0),
                                hrss=(1e-23, 1e-21))
# long-duration binary neutron stars: 256 s windows at 2048 Hz (N = 2^19),
# TaylorF2, Welch over the preceding 64 s (ranges: a reading)
CONFIGS["bns_long"] = dict(
    det_ids=(0, 1, 2), fs=2048.0, t_window=256.0, psd_length=64.0, fftlen=2.0, overlap=1.0,
    f_min=20.0, approximant=0, precision=1, mc=(1.0, 2.0), q=(0.5, 1.0), chi=(-0.05, 0.05),
    dl=(20.0, 300.0), batch=256, log2_bg=27)
# the shortest window: 2 s at 1024 Hz (N = 2048, a 1024-point window
# transform), otherwise the 64-signal TaylorF2 workload
CONFIGS["pr1_short"] = dict(CONFIGS["pr1_plain"], t_window=2.0)
CONFIGS["precision_study"] = dict(CONFIGS["paper_scale"], batch=8192)
CONFIGS["surrogate"] = dict(CONFIGS["paper_scale"], batch=8192)


# Uneven batches: 16384 signals, H1+L1+V1, durations {4, 8, 16} s x sample
# rates {1024, 2048} Hz (six classes), Welch over the 64 s before each window
# with 2 s segments at 50 % overlap; f_min 30 Hz for 4 s windows, else 20 Hz;
# priors of the paper-scale workload.  Each slot's class is drawn uniformly
# (seeded).
RAGGED_RATES = (1024.0, 2048.0)
RAGGED_DURATIONS = (4.0, 8.0, 16.0)
RAGGED_BATCH = 16384


def ragged_classes(precision=1):
    """The six class configurations, ordered (fs, T) = (1024, 4), (1024, 8),
    (1024, 16), (2048, 4), (2048, 8), (2048, 16)."""
    out = []
    for fs in RAGGED_RATES:
        for T in RAGGED_DURATIONS:
            c = dict(CONFIGS["paper_scale"], fs=fs, t_window=T, psd_length=64.0, fftlen=2.0, overlap=1.0,
                     f_min=30.0 if T == 4.0 else 20.0, precision=precision)
            c["log2_bg"] = 27 if fs == 2048.0 else 26
            out.append(c)
    return out


def ragged_assignment(B, n_classes=6, seed=11):
    """Class index per slot, uniform over the classes (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n_classes, size=B).astype(np.int32)


def config(name, **overrides):
    c = dict(CONFIGS[name])
    c.update(overrides)
    return c


def target_psd(f):
    f = np.maximum(np.asarray(f, dtype=np.float64), 10.0)
    x = f / 215.0
    return (2.0 ** 140) * 1e-49 * (x ** -4.14 - 5.0 * x ** -2
                                   + 111.0 * (1.0 - x * x + 0.5 * x ** 4)
                                   / (1.0 + 0.5 * x * x))


def colouring_fir(fs):
    M = int(round(4.0 * fs))
    f = np.arange(M // 2 + 1) * fs / M
    resp = np.sqrt(fs * target_psd(f) / 2.0)
    h = np.roll(np.fft.irfft(resp, n=M), M // 2)
    n = np.arange(M)
    return h * 0.5 * (1.0 - np.cos(2.0 * np.pi * n / M))


def true_psd(f, fs):
    """Exact one-sided PSD of the synthetic background at frequencies f."""
    h = colouring_fir(fs)
    f = np.atleast_1d(np.asarray(f, dtype=np.float64))
    n = np.arange(h.shape[0])
    out = np.empty_like(f)
    for i0 in range(0, f.shape[0], 512):
        ph = np.exp(-2j * np.pi * np.outer(f[i0:i0 + 512], n) / fs)
        out[i0:i0 + 512] = (2.0 / fs) * np.abs(ph @ h) ** 2
    return out


def background(n_det, length, fs, seed=1, dtype=np.float32, workers=None):
    """Coloured Gaussian background [n_det][length] (row d seeded seed*1000+d).

    A float32 request is coloured with single-precision transforms (its
    rounding, ~1e-7 relative, is far below the statistical scatter); float64
    uses double precision throughout.
    """
    import scipy.fft as sfft
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    h = colouring_fir(fs)
    if length < h.shape[0]:
        raise ValueError("background shorter than the colouring filter")
    single = np.dtype(dtype) == np.float32
    Hf = sfft.rfft(h, n=length, workers=workers)
    if single:
        Hf = Hf.astype(np.complex64)
    out = np.empty((n_det, length), dtype=dtype)
    for d in range(n_det):
        rng = np.random.Generator(np.random.PCG64(seed * 1000 + d))
        w = rng.standard_normal(length, dtype=np.float32 if single else np.float64)
        W = sfft.rfft(w, workers=workers)
        del w
        W *= Hf
        out[d] = sfft.irfft(W, n=length, workers=workers)
        del W
    return out


def white_background(n_det, length, sigma=1.0, seed=5, dtype=np.float32):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (sigma * rng.standard_normal((n_det, length))).astype(dtype)


def zero_background(n_det, length, dtype=np.float32):
    return np.zeros((n_det, length), dtype=dtype)


def bg_length_for(cfg, log2=None):
    """Default background length: 2**log2_bg samples (at least one stretch)."""
    lg = cfg.get("log2_bg", 22) if log2 is None else log2
    need = int(round((cfg["psd_length"] + cfg["t_window"]) * cfg["fs"]))
    return max(1 << lg, 1 << int(math.ceil(math.log2(need + 1))))
