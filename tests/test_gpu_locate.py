"""GPU parity of the FM-index intervals and of locate (the text positions of every occurrence, in
suffix-array order) against the oracle's suffix-array search, bit-exact: intervals equal the
oracle's SA ranges wherever a pattern occurs and are [0, 0) where it does not; locate's offsets
and positions equal the oracle's SA[lo..hi) per pattern, at several sampling rates (1, where every
row is sampled; small and large rates; a rate above n, where only the row of '$' is sampled)."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev
from tests.test_gpu_fm import csr, edge_patterns, make_text

pytestmark = pytest.mark.gpu


def check_intervals(fm, codes, sa, pat, off):
    dp, do = to_dev(pat if pat.size else np.zeros(1, np.uint8)), to_dev(off)
    iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32).astype(np.uint64)
    fm.check()
    lo, hi = oracle.interval_sa(codes, sa, pat, off)
    occ = hi > lo
    assert np.array_equal(iv[occ, 0], lo[occ]) and np.array_equal(iv[occ, 1], hi[occ])
    assert not iv[~occ].any()


def check_locate(fm, codes, sa, pat, off):
    dp, do = to_dev(pat if pat.size else np.zeros(1, np.uint8)), to_dev(off)
    start, pos = fm.locate(dp, do)
    fm.check()
    want_start, want_pos = oracle.locate_sa(codes, sa, pat, off)
    assert np.array_equal(start.cpu().numpy().view(np.uint64), want_start)
    assert np.array_equal(pos.cpu().numpy().view(np.uint32).astype(np.uint64), want_pos)


@pytest.mark.parametrize("n,rate", [(1, 1), (2, 4), (9, 1), (100, 3), (1000, 32), (65_537, 16), (65_537, 100_000)])
def test_intervals_and_locate_small(n, rate):
    qr = require_gpu()
    codes = make_text(50 + n, n)
    pats = edge_patterns(codes, 13 * n)
    sp, so, _ = datagen.patterns(n + 3, codes, 2000, minlen=1, maxlen=30, frac_sampled=0.8, sub=0.02)
    pats += [sp[int(so[i]):int(so[i + 1])] for i in range(so.size - 1)]
    pat, off = csr(pats)
    announce("fm-locate", n, rate, len(pats))
    fm = qr.QuadFm.from_text(codes, locate_rate=rate)
    sa = oracle.suffix_array(codes)
    check_intervals(fm, codes, sa, pat, off)
    check_locate(fm, codes, sa, pat, off)


def test_locate_medium_repeats():
    """2^20-base text with planted repeats (copies give intervals of about 20 rows); 2 x 10^4
    patterns of lengths 20..250 plus short patterns with many occurrences; rate 32."""
    qr = require_gpu()
    n = 1 << 20
    codes = make_text(91, n)
    pat, off, _ = datagen.patterns(93, codes, 20_000)
    short = [datagen.dna_codes(94 + k, 6 + k % 4) for k in range(50)]
    pats = [pat[int(off[i]):int(off[i + 1])] for i in range(off.size - 1)] + short
    pat, off = csr(pats)
    announce("fm-locate-medium", n)
    fm = qr.QuadFm.from_text(codes, locate_rate=32)
    sa = oracle.suffix_array(codes)
    check_intervals(fm, codes, sa, pat, off)
    check_locate(fm, codes, sa, pat, off)


def test_locate_repeated_calls_and_empty_batch():
    qr = require_gpu()
    n = 5000
    codes = make_text(7, n)
    announce("fm-locate-repeat")
    fm = qr.QuadFm.from_text(codes, locate_rate=8)
    sa = oracle.suffix_array(codes)
    pat, off = csr([codes[100:110], codes[:3], np.zeros(0, np.uint8)])
    for _ in range(2):
        check_locate(fm, codes, sa, pat, off)
    start, pos = fm.locate(to_dev(np.zeros(1, np.uint8)), to_dev(np.zeros(1, np.uint64)))
    assert start.cpu().numpy().tolist() == [0] and pos.numel() == 0


def test_locate_attach_rejects_bad_samples():
    qr = require_gpu()
    n = 3000
    codes = datagen.dna_codes(11, n)
    bwt, dollar, marks, samples = qr.quadfm_index_host(codes, 10)
    announce("fm-locate-attach-bad")
    fm = qr.QuadFm(torch.from_numpy(bwt.view(np.int64)).cuda(), n + 1, dollar)
    dm = torch.from_numpy(marks.view(np.int64)).cuda()
    with pytest.raises(qr.QRError):       # wrong number of samples for the rate
        fm.attach_locate(dm, torch.from_numpy(samples[:-1].view(np.int32)).cuda(), 10)
    bad = marks.copy()
    bad[dollar // 64] ^= np.uint64(1) << np.uint64(dollar % 64)   # unmark the row of '$'
    with pytest.raises(qr.QRError):
        fm.attach_locate(torch.from_numpy(bad.view(np.int64)).cuda(), torch.from_numpy(samples.view(np.int32)).cuda(), 10)
    with pytest.raises(qr.QRError):       # locate before any successful attach
        fm.locate(to_dev(codes[:5].copy()), to_dev(np.array([0, 5], np.uint64)))
    fm.attach_locate(dm, torch.from_numpy(samples.view(np.int32)).cuda(), 10)
    sa = oracle.suffix_array(codes)
    pat, off = csr([codes[7:12], codes[40:41]])
    check_locate(fm, codes, sa, pat, off)
