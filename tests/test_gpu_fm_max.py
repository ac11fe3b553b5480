"""The FM-index at its largest size: T = (ACGT)^k with n + 1 = 4k + 1 = 4294967293 BWT rows, just
under the 2^32 - 1 the build admits, so intervals, ranks and line indices reach the top of the
32-bit range the search works in.  The BWT of this text is known in closed form and so are the
counts, so no suffix array is built:
  - suffixes starting with a symbol sort by length (a shorter one meets '$' first);
  - so the rows are '$', then the k suffixes starting with A (preceded by T, except the whole text,
    preceded by '$'), then the C, G and T suffixes (preceded by A, C and G);
  - a pattern P occurs iff it is cyclic, P[i] = (s + i) mod 4, and then at the positions 4j + s with
    4j + s + |P| <= 4k."""
import numpy as np
import pytest

from tests.gpu_util import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu

K = 1073741823               # (ACGT)^K
N = 4 * K                    # text length
N1 = N + 1                   # BWT rows, <= 2^32 - 1
FILL = {0: 0x0, 1: 0x5555555555555555, 2: 0xAAAAAAAAAAAAAAAA, 3: 0xFFFFFFFFFFFFFFFF}


def packed_bwt():
    """2-bit packed BWT: rows [0, K) T, [K, 2K] A (row K is '$', stored as A), then K C and K G."""
    runs = [(0, K, 3), (K, 2 * K + 1, 0), (2 * K + 1, 3 * K + 1, 1), (3 * K + 1, N1, 2)]
    nw = (N1 + 31) // 32
    words = np.zeros(nw, dtype=np.uint64)
    for a, b, c in runs:
        w0, w1 = (a + 31) // 32, b // 32  # words lying wholly inside [a, b)
        if w0 < w1:
            words[w0:w1] = np.uint64(FILL[c])
    for a, b, c in runs:  # the words holding a run boundary, symbol by symbol
        for w in {a // 32, (b - 1) // 32}:
            for r in range(w * 32, min(w * 32 + 32, N1)):
                if a <= r < b:
                    words[w] = (words[w] & ~np.uint64(3 << (2 * (r % 32)))) | np.uint64(c << (2 * (r % 32)))
    return words


def cyclic_count(s, m):
    return max(0, (N - m - s) // 4 + 1) if m > 0 else N1


def pattern(s, m):
    return [(s + i) % 4 for i in range(m)]


def revcomp(p):
    return [3 - x for x in reversed(p)]


def is_cyclic(p):
    return all((p[i + 1] - p[i]) % 4 == 1 for i in range(len(p) - 1))


def expected(p):
    if not p:
        return N1
    return cyclic_count(p[0], len(p)) if is_cyclic(p) else 0


def csr(pats):
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in pats])
    flat = np.array([x for p in pats for x in p], np.uint8) if off[-1] else np.zeros(1, np.uint8)
    return flat, off


@pytest.mark.parametrize("kmer", [8, 12])
def test_fm_at_the_32_bit_limit(kmer):
    qr = require_gpu()
    announce("fm-max build", kmer, N1)
    fm = qr.QuadFm(to_dev(packed_bwt()), N1, K, kmer=kmer)
    c = fm.c_array()
    assert c.tolist() == [1, 1 + K, 1 + 2 * K, 1 + 3 * K]   # C[c] = 1 + #chars < c
    pats = [pattern(s, m) for s in range(4) for m in (1, 2, 3, 7, 8, 11, 12, 13, 20, 100, 250)]
    pats += [[0, 0], [0, 1, 2, 0], [3, 3, 3, 3], [2, 1], pattern(1, 12) + [0], [], pattern(3, 31) + [2]]
    flat, off = csr(pats)
    want = np.array([expected(p) for p in pats], np.uint32)
    announce("fm-max count", len(pats))
    dp, do = to_dev(flat), to_dev(off)
    got = fm.count(dp, do).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    got_b = fm.count_batched(dp, do, 7).cpu().numpy().view(np.uint32)
    assert np.array_equal(got_b, want)
    both = np.array([min(2 ** 32 - 1, expected(p) + expected(revcomp(p))) if p else N1 for p in pats], np.uint32)
    got_2 = fm.count(dp, do, both_strands=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(got_2, both)
    iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    size = np.where(iv[:, 1] > iv[:, 0], iv[:, 1] - iv[:, 0], 0)
    nonempty = np.array([len(p) > 0 for p in pats])
    assert np.array_equal(size[nonempty], want[nonempty].astype(np.int64))
    # single characters: the C-array buckets, the last one ending at the last row
    for s in range(4):
        i = pats.index(pattern(s, 1))
        assert tuple(iv[i]) == (int(c[s]), int(c[s]) + K)
    assert iv[pats.index(pattern(3, 1))][1] == N1
    fm.check()
