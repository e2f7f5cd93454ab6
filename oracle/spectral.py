"""Welch PSD, PSD interpolation and whitening (oracle side).

Section 3.2 of the paper fits the noise power spectrum to background strain
held on the accelerator and whitens every training window with it.  The
paper gives no estimator details; the readings used here:

  * one PSD per (sample, detector) from the P = psd_length * fs background
    samples immediately preceding that sample's window;
  * Welch's method: K = (P - L)/S + 1 segments of L = fftlen * fs samples at
    stride S = (fftlen - overlap) * fs, periodic Hann window
    w[n] = (1 - cos(2 pi n / L))/2, no detrending, mean over segments,
    one-sided density scaling
        S_hat[k] = (1/K) sum_s c_k |rfft(w * seg_s)[k]|^2 / (fs * sum w^2),
    c_k = 2 except at DC and Nyquist where c_k = 1;
  * interpolation onto the window grid (spacing 1/T) linearly in S with the
    integer ratio r = N / L;
  * whitening Y_k = rfft(y)_k / sqrt(fs * S_w[k] / 2) for f_k >= f_low and
    0 < k < N/2, zero elsewhere (also zero where S_w[k] is not a positive
    finite number); output irfft(Y).  No taper, no truncation.

Per-run mode (one PSD per detector for the whole run, then whitening with
a truncated inverse-spectrum filter):
  * run PSD: Welch as above over the first n_seg segments of the background
    row (the paper fits one spectrum to its background chunk);
  * the whitening gain g[k] above is turned into a finite impulse response
    of M taps: q = irfft_N(g), q_t[n] = q[n] cos^2(pi n / M) for |n| < M/2
    (n taken circularly in (-N/2, N/2]), 0 elsewhere; the filter is
    |rfft_N(q_t)| (the truncation smooths the gain; taking the magnitude
    drops the sign of the small negative ripples next to sharp cuts);
  * whitened output: irfft(rfft(y) * filter) with M/2 samples dropped at
    each end, where the filter's circular wrap-around reaches.

Pins: Welch equals scipy.signal.welch with the same settings; white noise
gives a flat PSD at 2 sigma^2/fs; noise with a known PSD whitened by that PSD
has variance 2 n_kept / N; a noise-free signal whitened by the true PSD has
squared norm equal to the optimal SNR^2.
"""

import numpy as np


def hann_periodic(L):
    n = np.arange(L, dtype=np.float64)
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * n / L))


def welch_psd(x, fs, L, S):
    """One-sided Welch PSD of the 1-D stretch x (len P) -> [L/2 + 1]."""
    x = np.asarray(x, dtype=np.float64)
    P = x.shape[0]
    if (P - L) % S:
        raise ValueError("stretch length is not a whole number of strides")
    K = (P - L) // S + 1
    w = hann_periodic(L)
    norm = fs * np.sum(w * w)
    acc = np.zeros(L // 2 + 1, dtype=np.float64)
    for s in range(K):
        X = np.fft.rfft(w * x[s * S:s * S + L])
        acc += np.abs(X) ** 2
    psd = acc / (K * norm)
    psd[1:L // 2] *= 2.0
    return psd


def interp_psd(psd, r):
    """Linear interpolation of an [L/2+1] PSD onto the [r*L/2+1] grid."""
    psd = np.asarray(psd, dtype=np.float64)
    n_out = (psd.shape[0] - 1) * r + 1
    j = np.arange(n_out)
    i = j // r
    t = (j % r) / r
    nxt = np.minimum(i + 1, psd.shape[0] - 1)
    return (1.0 - t) * psd[i] + t * psd[nxt]


def whiten(y, psd_w, fs, f_low):
    """Whiten the 1-D window y (len N) with the PSD psd_w on its rfft grid."""
    y = np.asarray(y, dtype=np.float64)
    N = y.shape[0]
    Y = np.fft.rfft(y)
    f = np.arange(N // 2 + 1) * fs / N
    psd_w = np.asarray(psd_w, dtype=np.float64)
    keep = (f >= f_low) & np.isfinite(psd_w) & (psd_w > 0.0)
    keep[0] = False
    keep[N // 2] = False
    out = np.zeros_like(Y)
    out[keep] = Y[keep] / np.sqrt(fs * psd_w[keep] / 2.0)
    return np.fft.irfft(out, n=N)


def whitening_gain(psd_w, fs, N, f_low):
    """g[k] = 1 / sqrt(fs S_w[k] / 2) on the kept bins, 0 elsewhere ([N/2+1])."""
    psd_w = np.asarray(psd_w, dtype=np.float64)
    f = np.arange(N // 2 + 1) * fs / N
    keep = (f >= f_low) & np.isfinite(psd_w) & (psd_w > 0.0)
    keep[0] = False
    keep[N // 2] = False
    g = np.zeros(N // 2 + 1)
    g[keep] = 1.0 / np.sqrt(fs * psd_w[keep] / 2.0)
    return g


def truncation_taper(N, M):
    """cos^2(pi n / M) for circular lags |n| < M/2, else 0 ([N])."""
    n = np.arange(N)
    n = np.where(n > N // 2, n - N, n)
    return np.where(np.abs(n) < M / 2.0, np.cos(np.pi * n / M) ** 2, 0.0)


def truncated_gain(psd_w, fs, N, f_low, M):
    """rfft_N of the tapered impulse response of the whitening gain (real)."""
    q = np.fft.irfft(whitening_gain(psd_w, fs, N, f_low), n=N)
    return np.real(np.fft.rfft(q * truncation_taper(N, M)))


def truncated_filter(psd_w, fs, N, f_low, M):
    """Whitening filter of the per-run mode: |truncated_gain| ([N/2+1])."""
    return np.abs(truncated_gain(psd_w, fs, N, f_low, M))


def whiten_filtered(y, filt, crop):
    """irfft(rfft(y) * filt) with `crop` samples dropped at each end."""
    y = np.asarray(y, dtype=np.float64)
    N = y.shape[0]
    out = np.fft.irfft(np.fft.rfft(y) * np.asarray(filt, dtype=np.float64), n=N)
    return out[crop:N - crop]


def run_psd(x, fs, L, S, n_seg):
    """Welch PSD over the first n_seg segments of the 1-D row x."""
    return welch_psd(np.asarray(x)[:(n_seg - 1) * S + L], fs, L, S)
