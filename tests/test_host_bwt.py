"""CPU parity of the product's host input preparation (SA-IS suffix array and BWT of T$, '$'
stored as A at its row) against the oracle's independent comparison-sort suffix array."""
import numpy as np
import pytest

import datagen
import oracle


def check_bwt(codes):
    import paper_2602_04103_amd as qr
    n = codes.size
    packed, dollar = qr.quadfm_bwt_host(codes)
    sa = oracle.suffix_array(codes)
    want, want_d = oracle.bwt(codes, sa)
    got = ((packed[np.arange(n + 1) // 32] >> (2 * (np.arange(n + 1) % 32)).astype(np.uint64)) & np.uint64(3))
    assert dollar == want_d
    w = want.astype(np.uint64)
    w[want_d] = 0  # '$' is stored as A
    assert np.array_equal(got, w)
    # bits beyond the last symbol are zero
    tail = (n + 1) % 32
    if tail:
        assert int(packed[-1]) >> (2 * tail) == 0


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 31, 32, 33, 100, 1000, 20000])
def test_bwt_random(n):
    check_bwt(datagen.dna_codes(1000 + n, n))


def test_bwt_repeats_and_degenerate():
    t = datagen.dna_codes(5, 60000)
    datagen.plant_repeats(6, t, nseg=10, seglen=2000, copies=5, sub=0.01)
    check_bwt(t)
    check_bwt(np.zeros(5000, np.uint8))
    check_bwt(np.full(3000, 3, np.uint8))
    check_bwt((np.arange(4097) % 4).astype(np.uint8))
    check_bwt((np.arange(5000) % 7 % 4).astype(np.uint8))
    check_bwt(np.tile(datagen.dna_codes(9, 37), 100))


def test_bwt_rejects_bad_codes():
    import paper_2602_04103_amd as qr
    with pytest.raises(qr.QRError):
        qr.quadfm_bwt_host(np.array([0, 1, 4, 2], np.uint8))


@pytest.mark.parametrize("n,rate", [(0, 1), (1, 1), (5, 2), (100, 7), (1000, 32), (20000, 32), (4097, 4096)])
def test_index_host_sa_sample(n, rate):
    """Mark bit k is set iff SA[k] is a multiple of rate, and the samples are SA of the marked rows in
    row order (oracle suffix array); the BWT is the same as without the sample."""
    import paper_2602_04103_amd as qr
    codes = datagen.dna_codes(2000 + n, n)
    if n >= 1000:
        datagen.plant_repeats(7, codes, nseg=3, seglen=200, copies=4, sub=0.01)
    packed, dollar, marks, samples = qr.quadfm_index_host(codes, rate)
    p2, d2 = qr.quadfm_bwt_host(codes)
    assert dollar == d2 and np.array_equal(packed, p2)
    sa = oracle.suffix_array(codes).astype(np.int64)
    bits = np.unpackbits(marks.view(np.uint8), bitorder="little")
    want = (sa % rate == 0)
    assert np.array_equal(bits[:n + 1].astype(bool), want)
    assert not bits[n + 1:].any()
    assert samples.size == n // rate + 1
    assert np.array_equal(samples.astype(np.int64), sa[want])
    assert bits[dollar] == 1                       # SA = 0 at the row of '$'
