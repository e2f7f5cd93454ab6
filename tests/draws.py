"""The oracle's own prior draws for the batch slots a GPU test checks.

Every GPU result compared with the oracle must be compared with what the
oracle computes from ITS inputs: the parameters and background offsets are
drawn here by the oracle (same Philox counters as the library) and the GPU's
draws are asserted equal to them (offsets bit-exact, parameters to 1e-12
relative) before the oracle's are used."""

import numpy as np

import oracle


def checked_draws(cfg, seed, first_index, P_gpu, O_gpu, L_bg, idx=None, ext_k=1):
    """(params, offsets) shaped like the GPU's, the columns idx (default all)
    drawn by the oracle at global index first_index + i; other columns are
    NaN / -1 so that using them by mistake fails."""
    P_gpu = np.asarray(P_gpu)
    O_gpu = np.asarray(O_gpu)
    B = P_gpu.shape[1]
    if idx is None:
        idx = range(B)
    idx = [int(i) for i in idx]
    P = np.full(P_gpu.shape, np.nan)
    O = np.full(O_gpu.shape, -1, dtype=np.int64)
    if len(idx) == B and idx == list(range(B)):
        p, o = oracle.sample_params(cfg, seed, first_index, B, L_bg, ext_k=ext_k)
        P[:], O[:] = p, o
    else:
        for i in idx:
            p, o = oracle.sample_params(cfg, seed, first_index + i, 1, L_bg, ext_k=ext_k)
            P[:, i], O[i] = p[:, 0], o[0]
    np.testing.assert_array_equal(O_gpu[idx], O[idx])
    np.testing.assert_allclose(P_gpu[:, idx], P[:, idx], rtol=1e-12, atol=1e-12)
    return P, O
