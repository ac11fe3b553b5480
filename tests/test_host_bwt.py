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
