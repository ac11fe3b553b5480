"""GPU parity of the FM-index over every QuadRank layout it runs on (the paper instantiates QuadFm
with each of its rank structures): the C array, the k-mer start table, counts from the persistent
and the per-batch kernels, both-strand counts, intervals and locate all equal the oracle's exactly
(u32, tolerance 0).  Small texts put the end of the text at every place of a line for the three
line payloads (384, 448 and 480 bases), one text crosses the first offset block of the paired
16-bit layout (122880 bases), and a 2^24-base text with repeats crosses every offset block of the
24/8 layout (2^15 lines = 12582912 bases) with 10^5 patterns checked against the oracle's
suffix-array search over an oracle-checked suffix array."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev
from tests.test_gpu_fm import csr, edge_patterns, make_text

pytestmark = pytest.mark.gpu

LAYOUT_NAMES = ("16", "16p", "32", "64", "24_8")


def layout_of(qr, name):
    return qr.LAYOUT_BY_NAME[name]


def check_all(qr, fm, codes, sa, pat, off, kmer):
    dp, do = to_dev(pat if pat.size else np.zeros(1, np.uint8)), to_dev(off)
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    assert np.array_equal(fm.count(dp, do).cpu().numpy().view(np.uint32), want)
    assert np.array_equal(fm.count_batched(dp, do, 333).cpu().numpy().view(np.uint32), want)
    both = oracle.count_both_strands(codes, sa, pat, off).astype(np.uint32)
    assert np.array_equal(fm.count(dp, do, both_strands=True).cpu().numpy().view(np.uint32), both)
    iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32).astype(np.uint64)
    lo, hi = oracle.interval_sa(codes, sa, pat, off)
    occ = hi > lo
    assert np.array_equal(iv[occ, 0], lo[occ]) and np.array_equal(iv[occ, 1], hi[occ])
    assert not iv[~occ].any()
    fm.check()
    cnt = np.bincount(codes, minlength=4).astype(np.uint64)
    assert np.array_equal(fm.c_array(), 1 + np.concatenate([[0], np.cumsum(cnt)[:3]]).astype(np.uint64))
    b, _ = oracle.bwt(codes, sa)
    klo, khi = oracle.kmer_intervals(b, kmer)
    tsp, tep = fm.table()
    nonempty = khi > klo
    assert np.array_equal(tsp[nonempty], klo[nonempty].astype(np.uint32))
    assert np.array_equal(tep[nonempty], khi[nonempty].astype(np.uint32))
    assert not np.any(tsp[~nonempty]) and not np.any(tep[~nonempty])


@pytest.mark.parametrize("layout", LAYOUT_NAMES)
@pytest.mark.parametrize("n", [1, 2, 9, 383, 385, 447, 449, 479, 481, 1000, 65_537, 130_001])
def test_fm_layout_small_texts(layout, n):
    qr = require_gpu()
    codes = make_text(300 + n, n)
    pats = edge_patterns(codes, 17 * n)
    sp, so, _ = datagen.patterns(n + 11, codes, 1500, minlen=1, maxlen=40, frac_sampled=0.8, sub=0.02)
    pats += [sp[int(so[i]):int(so[i + 1])] for i in range(so.size - 1)]
    pats += [oracle.revcomp(p) for p in pats[:30]]
    pat, off = csr(pats)
    kmer = 5 if n < 100_000 else 8
    announce("fm-layout", layout, n, len(pats))
    fm = qr.QuadFm.from_text(codes, locate_rate=4, kmer=kmer, layout=layout_of(qr, layout))
    assert qr.lib().quadfm_layout_kind(fm.h) == layout_of(qr, layout)
    sa = oracle.suffix_array(codes)
    check_all(qr, fm, codes, sa, pat, off, kmer)
    # locate: positions in suffix-array order
    dp, do = to_dev(pat if pat.size else np.zeros(1, np.uint8)), to_dev(off)
    start, pos = fm.locate(dp, do)
    fm.check()
    want_start, want_pos = oracle.locate_sa(codes, sa, pat, off)
    assert np.array_equal(start.cpu().numpy().view(np.uint64), want_start)
    assert np.array_equal(pos.cpu().numpy().view(np.uint32).astype(np.uint64), want_pos)
    fm.free()


def test_fm_layouts_2e24_with_repeats():
    """One BWT of 2^24 bases (200 planted 10-kb segments x 20 copies, 1% substitutions), prepared on
    the device with its suffix array handed out and checked by the oracle; every layout's index
    counts 10^5 patterns (lengths 20..250) exactly as the oracle's suffix-array search, with both
    kernels and both strands, sizes its intervals as counted, and counts 2*10^4 150-base reads (half
    reverse-complemented) on both strands from packed words as the oracle does."""
    qr = require_gpu()
    n = 1 << 24
    codes = datagen.dna_codes(2424, n)
    datagen.plant_repeats(2425, codes, nseg=200, seglen=10_000, copies=20, sub=0.01)
    pat, off, _ = datagen.patterns(2426, codes, 100_000)
    announce("fm-layouts 2^24 build")
    d_sa = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    bwt, dollar, _, _ = qr.quadfm_index_device(torch.from_numpy(codes).cuda(), 0, sa=d_sa)
    sa = d_sa.cpu().numpy().view(np.uint32).astype(np.int64)
    del d_sa
    assert oracle.check_sa(codes, sa) == 0
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    both = oracle.count_both_strands(codes, sa, pat[:int(off[10_000])], off[:10_001]).astype(np.uint32)
    dp, do = to_dev(pat), to_dev(off)
    # reads in the shape of the paper's experiment: 150 bases, 1 % substitutions, every other one
    # reverse-complemented, counted on both strands from 2-bit packed words
    rpat, roff, _ = datagen.patterns(2427, codes, 20_000, minlen=150, maxlen=150, frac_sampled=1.0, sub=0.01)
    rrows = rpat.reshape(-1, 150)
    rrows[1::2] = 3 - rrows[1::2, ::-1]
    rwant = oracle.count_both_strands(codes, sa, rpat, roff).astype(np.uint32)
    assert np.count_nonzero(rwant[0::2]) and np.count_nonzero(rwant[1::2])
    drp2, dro = to_dev(datagen.pack2(rpat)), to_dev(roff)
    sizes = {}
    for name in LAYOUT_NAMES:
        announce("fm-layouts 2^24", name)
        fm = qr.QuadFm(bwt, n + 1, dollar, kmer=10, layout=layout_of(qr, name))
        got = fm.count(dp, do).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), name
        assert np.array_equal(fm.count_batched(dp, do, 1 << 16).cpu().numpy().view(np.uint32), want), name
        g2 = fm.count(dp, do[:10_001], both_strands=True).cpu().numpy().view(np.uint32)
        assert np.array_equal(g2, both), name
        gr = fm.count_packed(drp2, rpat.size, dro, both_strands=True).cpu().numpy().view(np.uint32)
        assert np.array_equal(gr, rwant), name
        iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32).astype(np.int64)
        assert np.array_equal((iv[:, 1] - iv[:, 0]).astype(np.uint32), want), name
        fm.check()
        sizes[name] = fm.nbytes
        fm.free()
    # lines of 480, 480, 448, 384 and 384 bases: the index grows as the payload shrinks
    assert sizes["16p"] < sizes["16"] < sizes["32"] < sizes["64"]
    assert sizes["24_8"] > sizes["64"]  # the same lines plus an offset row per 2^15 lines


def test_fm_rejects_layout_without_one_lane_queries():
    qr = require_gpu()
    codes = datagen.dna_codes(5, 1000)
    bwt, d = qr.quadfm_bwt_host(codes)
    announce("fm-layout-reject")
    for bad in (qr.QR_LAYOUT_16X2, 7, -1):
        with pytest.raises(qr.QRError):
            qr.QuadFm(to_dev(bwt), 1001, d, layout=bad)
