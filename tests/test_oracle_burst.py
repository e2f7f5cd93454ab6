"""Pins of the sine-Gaussian burst model of the oracle: its closed-form
transform against a numerical transform of the time series, and its
normalisation (Parseval)."""

import math

import numpy as np
import pytest

from oracle import pipeline, priors, waveform
from paper_2407_19048_amd import inputs

S = waveform.STRAIN_SCALE


def _time_series(t, f0, Q, hrss, iota, phi0):
    tau = Q / (math.sqrt(2.0) * math.pi * f0)
    A = S * hrss / math.sqrt(tau * math.sqrt(math.pi / 2.0))
    env = np.exp(-(t / tau) ** 2)
    ci = math.cos(iota)
    hp = A * 0.5 * (1 + ci * ci) * env * np.cos(2 * math.pi * f0 * t + phi0)
    hc = A * ci * env * np.sin(2 * math.pi * f0 * t + phi0)
    return hp, hc


@pytest.mark.parametrize("f0,Q,iota,phi0", [(100.0, 5.0, 0.3, 1.1), (40.0, 3.0, 2.0, 4.0), (700.0, 25.0, 1.2, 0.2)])
def test_transform_matches_numerical_integral(f0, Q, iota, phi0):
    fs = 16384.0
    t = np.arange(-2.0, 2.0, 1.0 / fs)
    hp_t, hc_t = _time_series(t, f0, Q, 1e-22, iota, phi0)
    tau = Q / (math.sqrt(2.0) * math.pi * f0)
    f = np.array([0.3, 0.8, 1.0, 1.15, 1.6]) * f0
    assert tau > 0
    ker = np.exp(-2j * math.pi * np.outer(f, t)) / fs
    num_p, num_c = ker @ hp_t, ker @ hc_t
    hp, hc = waveform.sine_gaussian(f, f0, Q, 1e-22, iota, phi0, 0.0)
    scale = np.max(np.abs(hp))
    np.testing.assert_allclose(hp, num_p, atol=1e-9 * scale)
    np.testing.assert_allclose(hc, num_c, atol=1e-9 * scale)


def test_hrss_normalisation_parseval():
    f0, Q, hrss = 150.0, 9.0, 3e-22
    fs = 16384.0
    t = np.arange(-1.0, 1.0, 1.0 / fs)
    hp_t, hc_t = _time_series(t, f0, Q, hrss, 0.0, 0.7)
    e_time = np.sum(hp_t ** 2 + hc_t ** 2) / fs
    assert abs(e_time / (S * hrss) ** 2 - 1.0) < 1e-10
    f = np.arange(0.0, 4000.0, 0.05)
    hp, hc = waveform.sine_gaussian(f, f0, Q, hrss, 0.0, 0.7, 0.0)
    e_freq = 2.0 * np.sum(np.abs(hp) ** 2 + np.abs(hc) ** 2) * 0.05
    assert abs(e_freq / e_time - 1.0) < 1e-6


def test_burst_prior_rows():
    cfg = inputs.config("sine_gaussian")
    p, _ = priors.sample_params(cfg, 2, 0, 4000, 1 << 22)
    assert np.all((p[0] >= 32.0) & (p[0] < 1000.0))
    assert np.all((p[1] >= 3.0) & (p[1] < 30.0))
    lh = np.log10(p[2])
    assert np.all((lh >= -23.0) & (lh < -21.0))
    assert abs(np.mean(lh) + 22.0) < 0.05  # log-uniform
    assert np.all(p[3] == 0.0) and np.all(p[4] == 0.0)
    hp, hc = pipeline.waveform_on_grid(cfg, p[:, 0])
    assert hp[0] == 0 and hp[-1] == 0 and np.abs(hp).max() > 0
