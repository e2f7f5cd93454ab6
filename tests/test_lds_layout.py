"""Host model of the block FFT's LDS exchanges (no GPU): for every transform
size and pass order, every pass's reads and writes are free of bank conflicts
under the padding rule of the FFT header, the padded index of a split access
equals the padding of the whole index, and no index leaves the LDS buffer.

The bank model (32 banks of 4 bytes, a wave64 access served 32 lanes per
cycle) is the one a probe kernel measured with SQ_LDS_BANK_CONFLICT on the
target: it reproduced the measured conflict rate of every probe pattern
(contiguous runs, stride 16, groups of 16 and 32 at strides 256 and 512, pairs
at stride 32) for padding every 16, 32 and 64 words.  The plan and padding
constants below restate the header's (radix-16 passes, one small-radix pass
first or last; C = 1 for NS = 1 or NS >= 32, else 32/R)."""

import collections

import pytest

SIZES = (1024, 2048, 4096, 8192, 16384)


def plan(nc, order):
    np16 = 3 if nc >= 4096 else 2
    rl = nc // (4096 if np16 == 3 else 256)
    npass = np16 + (1 if rl > 1 else 0)
    out = []
    for p in range(npass):
        if order == 1 and rl > 1:
            r = rl if p == 0 else 16
            ns = 1 if p == 0 else rl * (1, 16, 256)[p - 1]
        else:
            r = 16 if p < np16 else rl
            ns = (1, 16, 256, 4096)[p]
        out.append((r, ns))
    return out


def pad_c(r, ns):
    return 1 if (ns == 1 or ns >= 32) else 32 // r


def xpad(i, c):
    return i + c * (i >> 5)


def worst_banks(indices):
    """Largest number of lanes of one 32-lane half that hit one bank."""
    w = 1
    for h in range(0, len(indices), 32):
        cnt = collections.Counter(i % 32 for i in indices[h:h + 32])
        w = max(w, max(cnt.values()))
    return w


def accesses(nc, order):
    """(padded read indices, padded write indices) per (pass, butterfly, element)."""
    nt = nc // 16
    pl = plan(nc, order)
    for p, (r, ns) in enumerate(pl):
        nb, stride = 16 // r, nc // r
        cr = 1 if p == 0 else pad_c(*pl[p - 1])
        cw = pad_c(r, ns)
        for m in range(nb):
            for e in range(r):
                reads = [xpad(t + nt * m + e * stride, cr) for t in range(nt)]
                writes = None
                if p < len(pl) - 1:
                    writes = []
                    for t in range(nt):
                        j = t + nt * m
                        k = j & (ns - 1)
                        writes.append(xpad((j - k) * r + k + e * ns, cw))
                yield p, reads, writes


@pytest.mark.parametrize("nc", SIZES)
@pytest.mark.parametrize("order", (0, 1))
def test_exchanges_conflict_free_and_in_bounds(nc, order):
    lds_words = nc + nc // 16
    for p, reads, writes in accesses(nc, order):
        assert worst_banks(reads) == 1, (nc, order, p, "read")
        assert max(reads) < lds_words
        if writes is not None:
            assert worst_banks(writes) == 1, (nc, order, p, "write")
            assert max(writes) < lds_words
            assert len(set(writes)) == len(writes)


@pytest.mark.parametrize("nc", SIZES)
@pytest.mark.parametrize("order", (0, 1))
def test_split_padding_is_exact(nc, order):
    """pad(base) + pad(offset) == pad(base + offset) for every split used."""
    nt = nc // 16
    pl = plan(nc, order)
    for p, (r, ns) in enumerate(pl):
        nb, stride = 16 // r, nc // r
        cr = 1 if p == 0 else pad_c(*pl[p - 1])
        cw = pad_c(r, ns)
        assert cw <= 2 and (ns == 1 or ns >= 32 or ns * r >= 32)
        for t in range(nt):
            for m in range(nb):
                j = t + nt * m
                k = j & (ns - 1)
                base = (j - k) * r + k
                for e in range(r):
                    assert xpad(j, cr) + xpad(e * stride, cr) == xpad(j + e * stride, cr)
                    assert xpad(base, cw) + xpad(e * ns, cw) == xpad(base + e * ns, cw)


def test_old_padding_conflicts_on_reads():
    """The model distinguishes: one pad word every 16 makes the contiguous
    reads 2-way conflicted (as measured before the change)."""
    reads = [t + 256 * 3 for t in range(256)]
    assert worst_banks([i + (i >> 4) for i in reads]) == 2
    assert worst_banks([xpad(i, 1) for i in reads]) == 1
