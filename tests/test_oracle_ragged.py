"""Pins of the oracle's uneven-batch definition: a slot is an ordinary sample
of its class, drawn at its global index, with the class index in row 11."""

import numpy as np

from oracle import pipeline, priors
from paper_2407_19048_amd import inputs


def _small_classes():
    # two of the six classes, shortened backgrounds (still several stretches)
    cl = inputs.ragged_classes()
    return [cl[0], cl[4]]  # (1024 Hz, 4 s) and (2048 Hz, 8 s)


def _bgs(classes):
    return [inputs.white_background(3, 1 << 18, seed=20 + k) for k, _ in enumerate(classes)]


def test_ragged_slot_equals_plain_sample_of_its_class():
    classes = _small_classes()
    bgs = _bgs(classes)
    cls = np.array([1, 0, 0, 1, 1], dtype=np.int32)
    seed, batch_index = 42, 3
    _, params, offs = pipeline.generate_ragged(classes, cls, seed, batch_index, bgs, slots=[])
    params, offs = pipeline.ragged_draws(classes, cls, seed, batch_index, [b.shape[1] for b in bgs])
    outs, p01, o01 = pipeline.generate_ragged(classes, cls, seed, batch_index, bgs, slots=[0, 1])
    np.testing.assert_array_equal(p01[:, :2], params[:, :2])
    np.testing.assert_array_equal(o01[:2], offs[:2])
    B = len(cls)
    for i in range(B):
        c = cls[i]
        p, o = priors.sample_params(classes[c], seed, batch_index * B, B, bgs[c].shape[1])
        np.testing.assert_array_equal(params[:11, i], p[:11, i])
        assert params[11, i] == float(c)
        assert offs[i] == o[i]
    for i in (0, 1):
        c = cls[i]
        ref = pipeline.generate_sample(classes[c], bgs[c], params[:, i], int(offs[i]))
        np.testing.assert_array_equal(outs[i], ref)
        assert outs[i].shape == (3, int(classes[c]["fs"] * classes[c]["t_window"]))


def test_ragged_class_recipe():
    cl = inputs.ragged_classes()
    sizes = [(c["fs"], c["t_window"], c["f_min"]) for c in cl]
    assert sizes == [(1024.0, 4.0, 30.0), (1024.0, 8.0, 20.0), (1024.0, 16.0, 20.0),
                     (2048.0, 4.0, 30.0), (2048.0, 8.0, 20.0), (2048.0, 16.0, 20.0)]
    for c in cl:
        z = pipeline.derived_sizes(c)
        assert z["K"] == 63 and z["N"] >= 2 * z["L"]
    a = inputs.ragged_assignment(16384)
    assert a.min() == 0 and a.max() == 5
    # mean bytes per sample of the recipe: 3 detectors x (P + N) read, N written
    rd = np.mean([3 * 4 * (pipeline.derived_sizes(c)["P"] + pipeline.derived_sizes(c)["N"]) for c in cl])
    assert rd == 1351680.0
