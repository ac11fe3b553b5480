"""GPU parity of the QuadFm count-only FM-index: counts from the persistent work-queue kernel and
from the one-launch-per-batch kernel equal the oracle's counts exactly (u32, tolerance 0); the C
array and the 8-mer interval table equal the oracle's textbook backward search."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def make_text(seed, n, repeats=True):
    codes = datagen.dna_codes(seed, n)
    if repeats and n >= 50_000:
        datagen.plant_repeats(seed + 1, codes, nseg=max(1, n // 100_000), seglen=min(10_000, n // 10), copies=20,
                              sub=0.01)
    return codes


def edge_patterns(codes, seed):
    n = codes.size
    pats = [np.zeros(0, np.uint8), codes[:1], codes[:7], codes[:8], codes[:9], codes[max(0, n - 8):],
            codes[max(0, n - 20):], codes.copy(), datagen.dna_codes(seed, n + 1), np.array([0, 1, 9, 2], np.uint8),
            np.array([1, 2, 3, 0, 1, 2, 3, 0, 7], np.uint8), np.array([5] + [0] * 10, np.uint8),
            np.array([2] * 12, np.uint8)]
    for k in range(1, 12):
        pats.append(datagen.dna_codes(seed + k, k))
    return pats


def csr(pats):
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in pats])
    flat = np.concatenate(pats).astype(np.uint8) if off[-1] else np.zeros(1, np.uint8)
    return flat, off


def gpu_counts(fm, pat, off, batch=None):
    dp, do = to_dev(pat if pat.size else np.zeros(1, np.uint8)), to_dev(off)
    if batch is None:
        c = fm.count(dp, do)
    else:
        c = fm.count_batched(dp, do, batch)
    fm.check()
    return c.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n", [1, 2, 9, 100, 1000, 65_537])
def test_fm_small_texts_all_kernels(n):
    qr = require_gpu()
    codes = make_text(40 + n, n)
    pats = edge_patterns(codes, 7 * n)
    sp, so, _ = datagen.patterns(n, codes, 2000, minlen=1, maxlen=40, frac_sampled=0.8, sub=0.02)
    pats += [sp[int(so[i]):int(so[i + 1])] for i in range(so.size - 1)]
    pat, off = csr(pats)
    announce("fm-small", n, len(pats))
    sa = oracle.suffix_array(codes)
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    for device_sa in (True, False):  # index input prepared on the device and on the host
        fm = qr.QuadFm.from_text(codes, device_sa=device_sa)
        assert np.array_equal(gpu_counts(fm, pat, off), want)
        assert np.array_equal(gpu_counts(fm, pat, off, batch=0), want)
        assert np.array_equal(gpu_counts(fm, pat, off, batch=333), want)


def test_fm_c_array_and_kmer_table():
    qr = require_gpu()
    n = 200_003
    codes = make_text(77, n)
    announce("fm-table", n)
    fm = qr.QuadFm.from_text(codes)
    cnt = np.bincount(codes, minlength=4).astype(np.uint64)
    want_C = 1 + np.concatenate([[0], np.cumsum(cnt)[:3]]).astype(np.uint64)
    assert np.array_equal(fm.c_array(), want_C)
    sa = oracle.suffix_array(codes)
    b, _ = oracle.bwt(codes, sa)
    lo, hi = oracle.kmer_intervals(b, 8)
    sp, ep = fm.table()
    nonempty = hi > lo
    assert np.array_equal(sp[nonempty], lo[nonempty].astype(np.uint32))
    assert np.array_equal(ep[nonempty], hi[nonempty].astype(np.uint32))
    assert np.all(sp[~nonempty] >= ep[~nonempty])


def test_fm_medium_random_patterns():
    """2^20-base text with planted repeats; 10^5 patterns of lengths 20..250 (90% sampled with 1%
    substitutions, 10% iid) — the batched configuration's distribution at a size the oracle's
    suffix-array search handles in seconds."""
    qr = require_gpu()
    n = 1 << 20
    codes = make_text(91, n)
    pat, off, kind = datagen.patterns(92, codes, 100_000)
    announce("fm-medium", n)
    fm = qr.QuadFm.from_text(codes)
    sa = oracle.suffix_array(codes)
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    got = gpu_counts(fm, pat, off)
    assert np.array_equal(got, want)
    assert np.array_equal(gpu_counts(fm, pat, off, batch=1 << 14), want)
    assert (want[kind == 1] > 0).mean() > 0.2   # exact copies occur; substituted ones mostly do not


@pytest.mark.parametrize("tune", [dict(refill=1), dict(refill=64), dict(refill=8, waves_per_cu=1),
                                  dict(block=64, refill=32, waves_per_cu=4), dict(waves_per_cu=32)])
def test_fm_persistent_tunings(tune):
    qr = require_gpu()
    n = 300_000
    codes = make_text(5, n)
    pat, off, _ = datagen.patterns(6, codes, 30_000)
    announce("fm-tune", tune)
    fm = qr.QuadFm.from_text(codes)
    fm.set_tuning(**tune)
    sa = oracle.suffix_array(codes)
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    for _ in range(2):  # the queue head is reset on every call
        assert np.array_equal(gpu_counts(fm, pat, off), want)


def test_fm_rejects_bad_dollar():
    qr = require_gpu()
    codes = datagen.dna_codes(3, 1000)
    bwt, d = qr.quadfm_bwt_host(codes)
    # claim '$' is at a row that holds a C/G/T: the build must refuse
    rows = (bwt[np.arange(1001) // 32] >> (2 * (np.arange(1001) % 32)).astype(np.uint64)) & np.uint64(3)
    bad = int(np.nonzero(rows != 0)[0][0])
    announce("fm-bad-dollar")
    with pytest.raises(qr.QRError):
        qr.QuadFm(to_dev(bwt), 1001, bad)
    with pytest.raises(qr.QRError):
        qr.QuadFm(to_dev(bwt), 1001, 1001)


def test_fm_config3_full():
    """Text of 2^28 bases with 1000 planted 10-kb repeats x 20 copies; 10^7 patterns (lengths
    20..250, 90% sampled with 1% substitutions, 10% iid).  The index input (suffix array, BWT and
    locate sample) is prepared on the device; its suffix array is handed out and checked by the
    oracle directly (a permutation whose neighbouring suffixes increase).  Every one of the 10^7
    persistent-kernel counts then equals the oracle's suffix-array binary search over the text, and
    so does every per-batch count, every count of the 2-bit packed patterns and every count of the
    same index over the other QuadRank layouts (16-bit paired, 32-bit, 64-bit and 24/8, with the
    12-mer start table); 10^5 150-base reads, half of them reverse-complemented, are counted on both
    strands as the oracle does.  200 sampled patterns are
    also recounted by the oracle's direct scan of the text.  Intervals and locate (SA sampled at rate
    32) are checked on the same index."""
    qr = require_gpu()
    n = 1 << 28
    codes = datagen.dna_codes(2028, n)
    datagen.plant_repeats(2029, codes, nseg=1000, seglen=10_000, copies=20, sub=0.01)
    pat, off, kind = datagen.patterns(2030, codes, 10 ** 7)
    announce("fm-config3 build")
    d_sa = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    bwt, dollar, marks, samples = qr.quadfm_index_device(torch.from_numpy(codes).cuda(), 32, sa=d_sa)
    fm = qr.QuadFm(bwt, n + 1, dollar)
    fm.attach_locate(marks, samples, 32)
    dp, do = to_dev(pat), to_dev(off)
    got_layouts = {}
    for name in ("16p", "32", "64", "24_8"):  # the same index over the other QuadRank layouts
        announce("fm-config3 count, layout", name)
        other = qr.QuadFm(bwt, n + 1, dollar, kmer=12, layout=qr.LAYOUT_BY_NAME[name])
        got_layouts[name] = other.count(dp, do).cpu().numpy().view(np.uint32)
        other.check()
        other.free()
    del bwt, marks, samples
    sa = d_sa.cpu().numpy().view(np.uint32).astype(np.int64)
    del d_sa
    announce("fm-config3 count")
    got = fm.count(dp, do).cpu().numpy().view(np.uint32)
    got_b = fm.count_batched(dp, do, 1 << 20).cpu().numpy().view(np.uint32)
    got_p = fm.count_packed(to_dev(datagen.pack2(pat)), int(off[-1]), do).cpu().numpy().view(np.uint32)
    # 10^5 reads of 150 bases with 1 % substitutions, every other one reverse-complemented, on both
    # strands from packed words (the shape of the paper's read-counting experiment)
    rpat, roff, _ = datagen.patterns(2831, codes, 100_000, minlen=150, maxlen=150, frac_sampled=1.0, sub=0.01)
    rrows = rpat.reshape(-1, 150)
    rrows[1::2] = 3 - rrows[1::2, ::-1]
    got_r = fm.count_packed(to_dev(datagen.pack2(rpat)), rpat.size, to_dev(roff),
                            both_strands=True).cpu().numpy().view(np.uint32)
    fm.check()
    announce("fm-config3 oracle: suffix-array check and 10^7 counts")
    assert oracle.check_sa(codes, sa) == 0
    want_all = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    assert np.array_equal(got, want_all)
    assert np.array_equal(got_b, want_all)
    assert np.array_equal(got_p, want_all)
    for name, g in got_layouts.items():
        assert np.array_equal(g, want_all), name
    want_r = oracle.count_both_strands(codes, sa, rpat, roff).astype(np.uint32)
    assert np.array_equal(got_r, want_r)
    assert np.count_nonzero(want_r[1::2]) > 0  # reverse-strand reads are found
    assert sa[dollar] == 0                       # the '$' row of the BWT is the row of suffix 0
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(10 ** 7, 200, replace=False))
    sp = [pat[int(off[i]):int(off[i + 1])] for i in sample]
    spat, soff = csr(sp)
    want = oracle.count_naive(codes, spat, soff).astype(np.uint32)
    assert np.array_equal(got[sample], want)
    assert got.max() <= n
    # intervals have the counted sizes; locate on the sample returns that many distinct positions,
    # each a true occurrence (so exactly the occurrence set), in suffix order
    iv_d = fm.intervals(dp, do)
    iv = iv_d.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal((iv[:, 1] - iv[:, 0]).astype(np.uint32), got)
    lo, hi = oracle.interval_sa(codes, sa, pat[:int(off[100_000])], off[:100_001])
    nz = hi > lo
    assert np.array_equal(iv[:100_000][nz, 0], lo[nz].astype(np.int64))   # intervals are the SA ranges
    # output offsets over all 10^7 intervals (thousands of scan tiles) = running sum of the counts
    st = torch.empty(10 ** 7 + 1, dtype=torch.int64, device="cuda")
    qr.quadfm_locate_offsets(fm.h, iv_d, st)
    want_st = np.concatenate([[0], np.cumsum(got.astype(np.uint64))]).astype(np.uint64)
    assert np.array_equal(st.cpu().numpy().view(np.uint64), want_st)
    announce("fm-config3 locate")
    start, pos = fm.locate(to_dev(spat), to_dev(soff))
    start, pos = start.cpu().numpy(), pos.cpu().numpy().view(np.uint32).astype(np.int64)
    w_start, w_pos = oracle.locate_sa(codes, sa, spat, soff)
    assert np.array_equal(start.astype(np.uint64), w_start)
    assert np.array_equal(pos.astype(np.uint64), w_pos)
    for k in range(len(sp)):
        ps = pos[start[k]:start[k + 1]]
        assert ps.size == want[k] and np.unique(ps).size == ps.size
        for x in ps:
            assert np.array_equal(codes[x:x + sp[k].size], sp[k])


@pytest.mark.parametrize("n", [3, 5000, 200_000])
def test_fm_both_strands(n):
    """count(P) + count(reverse complement of P), persistent and per-batch kernels."""
    qr = require_gpu()
    codes = make_text(600 + n, n)
    pats = edge_patterns(codes, 11 * n)
    sp, so, _ = datagen.patterns(n + 7, codes, 5000, minlen=1, maxlen=60, frac_sampled=0.8, sub=0.02)
    pats += [sp[int(so[i]):int(so[i + 1])] for i in range(so.size - 1)]
    pats += [oracle.revcomp(p) for p in pats[:50]]                 # palindromic and mirrored cases
    pat, off = csr(pats)
    announce("fm-both-strands", n, len(pats))
    fm = qr.QuadFm.from_text(codes)
    sa = oracle.suffix_array(codes)
    want = oracle.count_both_strands(codes, sa, pat, off).astype(np.uint32)
    dp, do = to_dev(pat), to_dev(off)
    got = fm.count(dp, do, both_strands=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    got_b = fm.count_batched(dp, do, 777, both_strands=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(got_b, want)


def test_fm_decreasing_offsets_count_zero_and_report():
    """A pattern whose offsets decrease is not read: it counts 0 (interval [0, 0)) and the sticky
    error reports it; the patterns around it are counted normally."""
    qr = require_gpu()
    codes = make_text(8, 5000)
    announce("fm-bad-offsets")
    fm = qr.QuadFm.from_text(codes)
    pat = codes[100:110].copy()
    off = np.array([0, 5, 3, 10], np.uint64)  # pattern 1 runs backwards
    want = oracle.count_naive(codes, pat, np.array([0, 5, 5, 10], np.uint64)).astype(np.uint32)
    want[1] = 0
    for kernel in ("persistent", "batched", "intervals"):
        dp, do = to_dev(pat), to_dev(off)
        if kernel == "persistent":
            got = fm.count(dp, do).cpu().numpy().view(np.uint32)
        elif kernel == "batched":
            got = fm.count_batched(dp, do, 2).cpu().numpy().view(np.uint32)
        else:
            iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32)
            got = (iv[:, 1] - iv[:, 0]).astype(np.uint32)
        want[2] = oracle.count_naive(codes, pat[3:10].copy(), np.array([0, 7], np.uint64))[0]
        assert np.array_equal(got, want), kernel
        with pytest.raises(qr.QRError) as ei:
            fm.check()
        assert ei.value.status == qr.QR_EINVAL
        fm.check()


def test_fm_offsets_past_pattern_buffer():
    """A pattern whose offsets run past the pattern buffer is not read: it counts 0 and the sticky
    error reports it, in every count form; with an empty pattern buffer (a NULL pointer and length
    0) only empty patterns are counted.  The length check happens before any pattern byte is
    loaded, so no launch here reads outside its buffers."""
    qr = require_gpu()
    codes = make_text(9, 5000)
    announce("fm-offsets-past-buffer")
    fm = qr.QuadFm.from_text(codes)
    pat = codes[200:230].copy()
    off = np.array([0, 10, 20, 30, 31, 1 << 40], np.uint64)   # patterns 3 and 4 end beyond 30 bytes
    good = oracle.count_naive(codes, pat, np.array([0, 10, 20, 30], np.uint64)).astype(np.uint32)
    want = np.concatenate([good, [0, 0]]).astype(np.uint32)
    dp, do = to_dev(pat), to_dev(off)
    for kernel in ("persistent", "batched", "both", "intervals"):
        if kernel == "persistent":
            got = fm.count(dp, do).cpu().numpy().view(np.uint32)
        elif kernel == "batched":
            got = fm.count_batched(dp, do, 2).cpu().numpy().view(np.uint32)
        elif kernel == "both":
            got = fm.count(dp, do, both_strands=True).cpu().numpy().view(np.uint32)
            w2 = oracle.count_both_strands(codes, oracle.suffix_array(codes), pat,
                                           np.array([0, 10, 20, 30], np.uint64)).astype(np.uint32)
            want = np.concatenate([w2, [0, 0]]).astype(np.uint32)
        else:
            iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32)
            got = (iv[:, 1] - iv[:, 0]).astype(np.uint32)
            want = np.concatenate([good, [0, 0]]).astype(np.uint32)
        assert np.array_equal(got, want), kernel
        with pytest.raises(qr.QRError) as ei:
            fm.check()
        assert ei.value.status == qr.QR_EINVAL
        fm.check()
    # an empty pattern buffer: the binding passes a NULL pointer with length 0
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    off2 = to_dev(np.array([0, 0, 4, 4], np.uint64))
    got = fm.count(empty, off2).cpu().numpy().view(np.uint32)
    assert got.tolist() == [codes.size + 1, 0, 0]   # [4, 4) lies past a buffer of 0 bytes as well
    with pytest.raises(qr.QRError):
        fm.check()
    fm.check()


def test_fm_plain_count_entry_point():
    """quadfm_count and quadfm_count_batched as the C ABI declares them (no buffer length), called
    directly: the same counts as the oracle on a well-formed CSR."""
    qr = require_gpu()
    import ctypes as C
    codes = make_text(12, 30_000)
    pat, off, _ = datagen.patterns(13, codes, 3000, minlen=1, maxlen=40, frac_sampled=0.8, sub=0.02)
    announce("fm-plain-entry")
    fm = qr.QuadFm.from_text(codes)
    want = oracle.count_sa(codes, oracle.suffix_array(codes), pat, off).astype(np.uint32)
    dp, do = to_dev(pat), to_dev(off)
    out = torch.empty(off.size - 1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert qr.lib().quadfm_count(C.c_void_p(fm.h), C.c_void_p(dp.data_ptr()), C.c_void_p(do.data_ptr()),
                                 C.c_uint64(off.size - 1), C.c_void_p(out.data_ptr()), C.c_void_p(s)) == 0
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
    out.zero_()
    assert qr.lib().quadfm_count_batched(C.c_void_p(fm.h), C.c_void_p(dp.data_ptr()), C.c_void_p(do.data_ptr()),
                                         C.c_uint64(off.size - 1), C.c_uint64(500), C.c_void_p(out.data_ptr()),
                                         C.c_void_p(s)) == 0
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
    fm.check()


@pytest.mark.parametrize("kmer", [1, 5, 10, 12])
def test_fm_start_table_sizes(kmer):
    """Start tables of other k: the table equals the oracle's k-mer intervals, and counts, both-strand
    counts and intervals equal the oracle's for patterns shorter and longer than k."""
    qr = require_gpu()
    n = 20_000 if kmer == 12 else 100_003
    codes = make_text(70 + kmer, n)
    pats = edge_patterns(codes, 3 * kmer)
    sp, so, _ = datagen.patterns(71 + kmer, codes, 3000, minlen=1, maxlen=40, frac_sampled=0.8, sub=0.02)
    pats += [sp[int(so[i]):int(so[i + 1])] for i in range(so.size - 1)]
    pat, off = csr(pats)
    announce("fm-kmer", kmer, n)
    fm = qr.QuadFm.from_text(codes, kmer=kmer)
    sa = oracle.suffix_array(codes)
    b, _ = oracle.bwt(codes, sa)
    lo, hi = oracle.kmer_intervals(b, kmer)
    tsp, tep = fm.table()
    nonempty = hi > lo
    assert np.array_equal(tsp[nonempty], lo[nonempty].astype(np.uint32))
    assert np.array_equal(tep[nonempty], hi[nonempty].astype(np.uint32))
    assert not np.any(tsp[~nonempty]) and not np.any(tep[~nonempty])
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    assert np.array_equal(gpu_counts(fm, pat, off), want)
    assert np.array_equal(gpu_counts(fm, pat, off, batch=1000), want)
    dp, do = to_dev(pat), to_dev(off)
    both = fm.count(dp, do, both_strands=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(both, oracle.count_both_strands(codes, sa, pat, off).astype(np.uint32))
    iv = fm.intervals(dp, do).cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal((iv[:, 1] - iv[:, 0]).astype(np.uint32), want)
    fm.check()


def test_fm_rejects_bad_kmer():
    qr = require_gpu()
    codes = datagen.dna_codes(3, 1000)
    announce("fm-bad-kmer")
    for k in (0, 13):
        with pytest.raises(qr.QRError):
            qr.QuadFm.from_text(codes, kmer=k)


@pytest.mark.parametrize("layout", ["16", "32"])
@pytest.mark.parametrize("n", [1, 1000, 200_000])
def test_fm_count_packed(layout, n):
    """Counts over 2-bit packed patterns (one stream of u64 words, offsets in bases) equal the
    byte-pattern counts and the oracle's, one strand and both: patterns start at every place of a
    word (a filler of k bases precedes them), span several words, are empty or shorter than the
    start table, and the stream's last word carries garbage past its last base.  A pattern whose
    offsets run past the stream's length counts 0 and is reported."""
    qr = require_gpu()
    codes = make_text(900 + n, n)
    pats = [p for p in edge_patterns(codes, 19 * n) if p.size == 0 or p.max() <= 3]
    sp, so, _ = datagen.patterns(n + 13, codes, 3000, minlen=1, maxlen=120, frac_sampled=0.8, sub=0.02)
    pats += [sp[int(so[i]):int(so[i + 1])] for i in range(so.size - 1)]
    pats += [oracle.revcomp(p) for p in pats[:40]]
    pat, off = csr(pats)
    announce("fm-packed", layout, n, len(pats))
    fm = qr.QuadFm.from_text(codes, kmer=8, layout=qr.LAYOUT_BY_NAME[layout])
    sa = oracle.suffix_array(codes)
    want = oracle.count_sa(codes, sa, pat, off).astype(np.uint32)
    both = oracle.count_both_strands(codes, sa, pat, off).astype(np.uint32)
    total = int(off[-1])
    for k in (0, 1, 17, 31, 32, 45):  # filler bases before the first pattern
        stream = np.concatenate([datagen.dna_codes(7 + k, k), pat[:total]]).astype(np.uint8)
        words = to_dev(datagen.pack2(stream, tail_garbage=True, seed=k + 1))
        o = to_dev((off + np.uint64(k)).astype(np.uint64))
        got = fm.count_packed(words, stream.size, o).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), k
        got2 = fm.count_packed(words, stream.size, o, both_strands=True).cpu().numpy().view(np.uint32)
        assert np.array_equal(got2, both), k
        fm.check()
    # offsets past the stream: counted 0, reported, nothing read beyond it
    words = to_dev(datagen.pack2(pat[:total] if total else np.zeros(1, np.uint8)))
    bad = off.copy()
    bad[-1] = total + 64
    got = fm.count_packed(words, total, to_dev(bad)).cpu().numpy().view(np.uint32)
    assert got[-1] == 0 and np.array_equal(got[:-1], want[:-1])
    with pytest.raises(qr.QRError):
        fm.check()
    fm.free()
