"""Counter-based random numbers for the prior draws (oracle side).

The paper does not say how its prior draws are generated.  The generator is
Philox4x32-10 from Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11), written here with plain Python integers from that
definition.  The HIP side carries its own implementation; the two agree bit
for bit, and this one is pinned to the published known-answer vectors.

Counter layout for prior draws: key = (seed & 0xffffffff, seed >> 32),
counter = (index & 0xffffffff, index >> 32, stream, sub), where index is the
global sample index (batch_index * B + i), so a run's output does not depend
on how it is split into batches.  sub is 0 except for the extrinsic draws of
oversampled batches (the j-th sky position of an intrinsic draw uses j).

Uniform in the open interval (0, 1) from the first two output words a, b:
u = ((a >> 5) * 2**26 + (b >> 6) + 0.5) * 2**-53, exact in binary64.
"""

MASK32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def _round(ctr, key):
    c0, c1, c2, c3 = ctr
    p0 = PHILOX_M0 * c0
    p1 = PHILOX_M1 * c2
    hi0, lo0 = p0 >> 32, p0 & MASK32
    hi1, lo1 = p1 >> 32, p1 & MASK32
    return (hi1 ^ c1 ^ key[0], lo1, hi0 ^ c3 ^ key[1], lo0)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds; ctr is four 32-bit words, key two."""
    ctr = tuple(int(c) & MASK32 for c in ctr)
    key = [int(k) & MASK32 for k in key]
    for r in range(10):
        if r:
            key = [(key[0] + PHILOX_W0) & MASK32, (key[1] + PHILOX_W1) & MASK32]
        ctr = _round(ctr, key)
    return ctr


def philox_uniform(seed, index, stream, sub=0):
    """One binary64 uniform in (0, 1) for (seed, global sample index, stream, sub)."""
    seed = int(seed)
    index = int(index)
    a, b, _, _ = philox4x32_10(
        (index & MASK32, (index >> 32) & MASK32, int(stream), int(sub)),
        (seed & MASK32, (seed >> 32) & MASK32))
    return ((a >> 5) * 67108864 + (b >> 6) + 0.5) * 2.0 ** -53


def philox_uniforms(seed, first_index, count, stream):
    """`count` uniforms for consecutive global indices starting at first_index."""
    import numpy as np
    return np.array([philox_uniform(seed, first_index + i, stream)
                     for i in range(count)], dtype=np.float64)
