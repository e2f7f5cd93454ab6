"""Pins of the oracle's view pairs and extrinsic oversampling."""

import math

import numpy as np
from scipy import stats

from oracle import pipeline, priors
from paper_2407_19048_amd import inputs


def _cfg():
    return inputs.config("pr1_plain")


def test_oversampling_with_k_1_is_the_ordinary_draw():
    cfg = _cfg()
    p1, o1 = priors.sample_params(cfg, 3, 40, 6, 1 << 20)
    pk, ok = priors.sample_params(cfg, 3, 40, 6, 1 << 20, ext_k=1)
    np.testing.assert_array_equal(p1, pk)
    np.testing.assert_array_equal(o1, ok)


def test_oversampled_groups_share_intrinsic_rows_only():
    cfg = _cfg()
    k, B = 4, 12
    p, o = priors.sample_params(cfg, 5, 8, B, 1 << 20, ext_k=k)  # global 8..19: draws 2..4
    plain, plain_o = priors.sample_params(cfg, 5, 2, 3, 1 << 20)
    shared = [0, 1, 2, 3, 4, 5, 9, 10]
    for grp in range(3):
        cols = slice(grp * k, (grp + 1) * k)
        for r in shared:
            assert np.all(p[r, cols] == plain[r, grp])
        for r in (6, 7, 8):
            assert len(set(p[r, cols])) == k
        assert len(set(o[cols])) == k
        # sky position 0 of a draw is the ordinary draw
        np.testing.assert_array_equal(p[:, grp * k], plain[:, grp])
        assert o[grp * k] == plain_o[grp]


def test_oversampled_sky_positions_follow_the_priors():
    cfg = _cfg()
    p, _ = priors.sample_params(cfg, 11, 0, 2000, 1 << 20, ext_k=8)
    assert stats.kstest(p[6] / (2 * math.pi), "uniform").pvalue > 1e-3
    assert stats.kstest((np.sin(p[7]) + 1) / 2, "uniform").pvalue > 1e-3
    assert stats.kstest(p[8] / math.pi, "uniform").pvalue > 1e-3


def test_reference_view_is_the_shifted_view_moved_by_the_delay():
    """Whitening is a circular filter, and a t_c change of n samples is a
    circular shift of the signal by n: the whitened signals of the two views
    differ by exactly that shift."""
    cfg = _cfg()
    z = pipeline.derived_sizes(cfg)
    fs = float(cfg["fs"])
    bg = inputs.white_background(2, 1 << 17, sigma=1.0, seed=2).astype(np.float64)
    p, o = priors.sample_params(cfg, 4, 0, 1, bg.shape[1])
    p = p[:, 0].copy()
    n = 300
    p[10] = pipeline.reference_time(cfg) + n / fs
    d_ref, d_shift = pipeline.generate_pair(cfg, bg, p, int(o[0]))
    quiet = p.copy()
    quiet[4] = 1e30  # no signal: the whitened noise alone
    noise = pipeline.generate_sample(cfg, bg, quiet, int(o[0]))
    w_ref, w_shift = d_ref - noise, d_shift - noise
    assert np.linalg.norm(w_ref) > 1e-3 * np.linalg.norm(noise)
    np.testing.assert_allclose(w_shift, np.roll(w_ref, n, axis=1), atol=1e-9 * np.abs(w_ref).max())
    assert z["N"] == d_ref.shape[1]
