"""Pins of the per-run PSD mode of the oracle: one Welch PSD per detector for
the run, a truncated (tapered, finite impulse response) whitening filter and
cropped whitened windows."""

import numpy as np
import pytest
from scipy import signal

from oracle import pipeline, spectral


def test_taper_is_periodic_hann_centred_at_lag_zero():
    N, M = 64, 16
    h = spectral.truncation_taper(N, M)
    ref = np.zeros(N)
    ref[np.arange(-M // 2, M // 2) % N] = signal.windows.hann(M, sym=False)
    np.testing.assert_allclose(h, ref, atol=1e-15)


def test_run_psd_equals_library_welch_and_chunk_means():
    rs = np.random.default_rng(0)
    fs, L, S, K = 256.0, 64, 32, 7
    n_chunks = 5
    x = rs.standard_normal(n_chunks * K * S + L + 100)
    got = spectral.run_psd(x, fs, L, S, n_chunks * K)
    n = (n_chunks * K - 1) * S + L
    _, ref = signal.welch(x[:n], fs=fs, window="hann", nperseg=L, noverlap=L - S, detrend=False,
                          scaling="density", average="mean")
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    # the mean of per-chunk Welch PSDs (K segments each, chunk c starting at
    # segment c K) is the same estimate
    P = (K - 1) * S + L
    chunks = [spectral.welch_psd(x[c * K * S:c * K * S + P], fs, L, S) for c in range(n_chunks)]
    np.testing.assert_allclose(np.mean(chunks, axis=0), got, rtol=1e-12)


def _smooth_psd(f):
    return 1e-2 * (1.0 + (f / 40.0) ** 2) / (1.0 + (f / 300.0) ** 4)


@pytest.mark.parametrize("f_low", [0.0, 20.0])
def test_truncated_gain_has_the_tapered_response(f_low):
    fs, N, M = 1024.0, 4096, 1024
    f = np.arange(N // 2 + 1) * fs / N
    S = _smooth_psd(f)
    tg = spectral.truncated_gain(S, fs, N, f_low, M)
    q = np.fft.irfft(tg, n=N)
    lag = np.arange(N)
    lag = np.where(lag > N // 2, lag - N, lag)
    inside = np.abs(lag) < M // 2
    full = np.fft.irfft(spectral.whitening_gain(S, fs, N, f_low), n=N)
    scale = np.max(np.abs(full))
    assert np.max(np.abs(q[~inside])) < 1e-12 * scale
    np.testing.assert_allclose(q[inside], full[inside] * np.cos(np.pi * lag[inside] / M) ** 2,
                               atol=1e-12 * scale)
    filt = spectral.truncated_filter(S, fs, N, f_low, M)
    np.testing.assert_array_equal(filt, np.abs(tg))


def test_truncated_filter_approaches_the_gain_for_a_smooth_spectrum():
    fs, N = 1024.0, 8192
    f = np.arange(N // 2 + 1) * fs / N
    S = _smooth_psd(f)
    g = spectral.whitening_gain(S, fs, N, 0.0)
    filt = spectral.truncated_filter(S, fs, N, 0.0, N // 2)
    band = slice(20, N // 2 - 20)
    err = np.linalg.norm(filt[band] - g[band]) / np.linalg.norm(g[band])
    assert err < 2e-3


def test_noise_whitened_with_the_truncated_filter_has_unit_variance():
    rs = np.random.default_rng(3)
    fs, N, M = 1024.0, 16384, 2048
    f = np.arange(N // 2 + 1) * fs / N
    S = _smooth_psd(f)
    # circular noise with one-sided PSD S: rfft amplitudes sqrt(fs N S / 4) per component
    outs = []
    for _ in range(8):
        Z = (rs.standard_normal(N // 2 + 1) + 1j * rs.standard_normal(N // 2 + 1)) * np.sqrt(fs * N * S / 4.0)
        Z[0] = Z[0].real * np.sqrt(2.0)
        Z[-1] = Z[-1].real * np.sqrt(2.0)
        y = np.fft.irfft(Z, n=N)
        filt = spectral.truncated_filter(S, fs, N, 0.0, M)
        outs.append(spectral.whiten_filtered(y, filt, M // 2))
    var = np.var(np.concatenate(outs))
    assert abs(var - 1.0) < 0.02


def test_runpsd_sample_equals_plain_whitening_without_truncation_effects():
    """With the sample's own PSD and a filter that keeps all N taps but the
    last, the per-run path reduces to the plain whitening up to the taper."""
    cfg = dict(det_ids=(0,), fs=256.0, t_window=8.0, psd_length=16.0, fftlen=2.0, overlap=1.0,
               f_min=0.0, approximant=0, precision=1, mc=(10.0, 20.0), q=(0.5, 1.0), chi=(0.0, 0.0),
               dl=(100.0, 200.0))
    z = pipeline.derived_sizes(cfg)
    rs = np.random.default_rng(5)
    bg = rs.standard_normal((1, 1 << 14))
    psd = pipeline.run_psds(cfg, bg, 4)
    assert psd.shape == (1, z["Fw"])
    filt = pipeline.run_filters(cfg, psd, 64)
    assert filt.shape == (1, z["F"])
    g = spectral.whitening_gain(spectral.interp_psd(psd[0], z["r"]), cfg["fs"], z["N"], 0.0)
    # a 64-tap filter still follows the gain's broad shape
    band = slice(8, z["F"] - 8)
    assert np.linalg.norm(filt[0][band] - g[band]) / np.linalg.norm(g[band]) < 0.2
