"""GPU parity of the layout variants against the oracle, bit-exact (tolerance 0): paired
superblocks (the paper's appendix on pairing superblocks) for BiRank and QuadRank, the 64-bit
absolute layouts BiRank64 and QuadRank64, BiRank16x2 (Section 3 "Variants") and QuadRank24_8
(Section 4 "Variants"), each re-derived for 128-byte lines.  For every layout: an edge battery of
sizes around line, build-group, superblock, pair-middle and anchor boundaries with garbage tail
bits, constant and degenerate inputs, every query-kernel tuning (one lane, lane pairs, sweep tiles),
out-of-range queries, and a structure decoder that checks every stored delta and offset against
the oracle's rank at the position the layout defines."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import announce, edge_queries, require_gpu, to_dev, to_host_u64
from tests.test_gpu_rank import TUNINGS, qr_text

pytestmark = pytest.mark.gpu

SWEEP_TUNINGS = [dict(lanes=2, per_lane=1, sweep=1024), dict(lanes=2, per_lane=2, sweep=4096),
                 dict(lanes=2, per_lane=1, sweep=2048)]

# BiRank layouts: (name, data bits per line, anchor data positions, lines per offset entry)
BR_GEOM = {
    "16p": (1008, (496,), 128),
    "64": (960, (448,), None),
    "16x2": (992, (224, 736), 64),
}


def br_layout(qr, name):
    return {"16p": qr.QR_LAYOUT_16P, "64": qr.QR_LAYOUT_64, "16x2": qr.QR_LAYOUT_16X2}[name]


def br_sizes(name):
    line, _, sb = BR_GEOM[name]
    sb_bits = (sb or 128) * line
    return [0, 1, 63, 64, 65, line - 1, line, line + 1, 64 * line - 1, 64 * line, 64 * line + 1, sb_bits - 1, sb_bits,
            sb_bits + 1, 3 * sb_bits + 64 * line + 7, (1 << 20) + 17]


def br_queries(name, n, seed, k=20000):
    line, anchors, sb = BR_GEOM[name]
    parts = [datagen.queries(seed, n, k)]
    for a in anchors:
        parts.append(edge_queries(n, line, a, (sb or 128) * line))
    parts.append(edge_queries(n, line, anchors[0], 64 * line))         # pair middles and group starts
    if n <= 70000:
        parts.append(np.arange(n + 1, dtype=np.uint64))
    return np.unique(np.concatenate(parts))


@pytest.mark.parametrize("p", [0.5, 0.05])
@pytest.mark.parametrize("name,n", [(nm, n) for nm in BR_GEOM for n in br_sizes(nm)])
def test_birank_variant_edge_battery(name, n, p):
    qr = require_gpu()
    bits = datagen.bits(1700 + n, n, p, tail_garbage=True)
    q = br_queries(name, n, 500 + n)
    announce("birank-variant", name, n, p, q.size)
    br = qr.BiRank(to_dev(bits), n, layout=br_layout(qr, name))
    assert qr.lib().birank_layout_kind(br.h) == br_layout(qr, name)
    want = oracle.rank_bits(bits, n, q)
    for tune in (dict(), dict(lanes=1), dict(lanes=2, per_lane=1, sweep=1024)):
        br.set_tuning(**tune)
        assert np.array_equal(to_host_u64(br.rank(to_dev(q))), want), (name, tune)
    br.check()


@pytest.mark.parametrize("name", list(BR_GEOM))
@pytest.mark.parametrize("fill", [0, 1])
def test_birank_variant_constant_bitvectors(name, fill):
    qr = require_gpu()
    line, _, sb = BR_GEOM[name]
    n = 5 * (sb or 128) * line + 777
    bits = np.full((n + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF) if fill else np.uint64(0))
    q = br_queries(name, n, 3)
    announce("birank-variant-constant", name, fill)
    got = to_host_u64(qr.BiRank(to_dev(bits), n, layout=br_layout(qr, name)).rank(to_dev(q)))
    assert np.array_equal(got, q if fill else np.zeros_like(q))


@pytest.mark.parametrize("name", list(BR_GEOM))
@pytest.mark.parametrize("tune", TUNINGS + SWEEP_TUNINGS)
def test_birank_variant_tunings(name, tune):
    qr = require_gpu()
    line, _, sb = BR_GEOM[name]
    n = 3 * (sb or 128) * line + 4321
    bits = datagen.bits(199, n, 0.5)
    q = np.concatenate([br_queries(name, n, 198), datagen.queries(197, n, 100_003)])
    announce("birank-variant-tune", name, tune)
    br = qr.BiRank(to_dev(bits), n, layout=br_layout(qr, name))
    br.set_tuning(**tune)
    assert np.array_equal(to_host_u64(br.rank(to_dev(q))), oracle.rank_bits(bits, n, q))


@pytest.mark.parametrize("name", list(BR_GEOM))
def test_birank_variant_out_of_range(name):
    qr = require_gpu()
    n = 5000
    bits = datagen.bits(1, n)
    q = np.array([0, n, n + 1, 2 ** 63, 17], dtype=np.uint64)
    announce("birank-variant-out-of-range", name)
    br = qr.BiRank(to_dev(bits), n, layout=br_layout(qr, name))
    assert np.array_equal(to_host_u64(br.rank(to_dev(q))), oracle.rank_bits(bits, n, q))
    with pytest.raises(qr.QRError):
        br.check()
    br.check()


def _bits_of_lines(lines):
    nl = lines.shape[0]
    return np.unpackbits(lines.view(np.uint8), bitorder="little").reshape(nl, 1024)


def test_birank16p_structure_decoder():
    """Paired superblocks: s'_i = floor(rank(1008 (128 i + 64)) / 2^10) (the rank at the pair's
    middle, over the zero-padded bits); each line's delta minus BIAS = 64*1008 - 496 for the lower
    64 lines of a pair, plus 2^10 s', is the oracle rank at the line's middle; data round-trips."""
    qr = require_gpu()
    n = 7 * 129024 + 64512 + 1234
    bits = datagen.bits(4242, n, 0.5, tail_garbage=True)
    announce("birank16p-structure", n)
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_16P)
    lines, sup = br.export()
    nl = lines.shape[0]
    assert nl == n // 1008 + 1 and sup.size == (nl - 1) // 128 + 1 and sup.dtype == np.uint32
    i = np.arange(sup.size, dtype=np.uint64)
    pair_mid = np.minimum(1008 * (128 * i + 64), n).astype(np.uint64)
    assert np.array_equal(sup.astype(np.uint64), oracle.rank_bits(bits, n, pair_mid) >> np.uint64(10))
    j = np.arange(nl, dtype=np.uint64)
    b = (lines[:, 0] & np.uint64(0xFFFF)).astype(np.int64)
    lower = (j % np.uint64(128)) < np.uint64(64)
    anchor = (sup[(j // np.uint64(128)).astype(np.int64)].astype(np.int64) << 10) + b - np.where(lower, 64 * 1008 - 496, 0)
    want = oracle.rank_bits(bits, n, np.minimum(j * np.uint64(1008) + np.uint64(496), n).astype(np.uint64))
    assert np.array_equal(anchor.astype(np.uint64), want)
    assert (b[lower] <= 64 * 1008 - 496 + 1023).all()
    lb = _bits_of_lines(lines)[:, 16:].reshape(-1)
    ib = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    assert np.array_equal(lb[:n], ib) and not lb[n:].any()


def test_birank64_structure_decoder():
    """BiRank64: the first 64 bits of line j are the oracle rank at data bit 960 j + 448; no offsets."""
    qr = require_gpu()
    n = 9 * 61440 + 4321
    bits = datagen.bits(4343, n, 0.5, tail_garbage=True)
    announce("birank64-structure", n)
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_64)
    lines, sup = br.export()
    nl = lines.shape[0]
    assert nl == n // 960 + 1 and sup.size == 0 and br.nbytes == nl * 128
    j = np.arange(nl, dtype=np.uint64)
    want = oracle.rank_bits(bits, n, np.minimum(j * np.uint64(960) + np.uint64(448), n).astype(np.uint64))
    assert np.array_equal(lines[:, 0], want)
    lb = _bits_of_lines(lines)[:, 64:].reshape(-1)
    ib = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    assert np.array_equal(lb[:n], ib) and not lb[n:].any()


def test_birank16x2_structure_decoder():
    """BiRank16x2: the two 16-bit deltas of line j plus 2^10 s_{j/64} are the oracle ranks at data
    bits 992 j + 224 and 992 j + 736 (line bits 256 and 768); s_i = floor(rank(63488 i) / 2^10)."""
    qr = require_gpu()
    n = 6 * 63488 + 777
    bits = datagen.bits(4444, n, 0.5, tail_garbage=True)
    announce("birank16x2-structure", n)
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_16X2)
    lines, sup = br.export()
    nl = lines.shape[0]
    assert nl == n // 992 + 1 and sup.size == (nl - 1) // 64 + 1
    i = np.arange(sup.size, dtype=np.uint64)
    assert np.array_equal(sup.astype(np.uint64),
                          oracle.rank_bits(bits, n, np.minimum(i * np.uint64(63488), n).astype(np.uint64)) >> np.uint64(10))
    j = np.arange(nl, dtype=np.uint64)
    off = sup[(j // np.uint64(64)).astype(np.int64)].astype(np.uint64) << np.uint64(10)
    for shift, a in ((0, 224), (16, 736)):
        d = (lines[:, 0] >> np.uint64(shift)) & np.uint64(0xFFFF)
        want = oracle.rank_bits(bits, n, np.minimum(j * np.uint64(992) + np.uint64(a), n).astype(np.uint64))
        assert np.array_equal(off + d, want), a
    lb = _bits_of_lines(lines)[:, 32:].reshape(-1)
    ib = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    assert np.array_equal(lb[:n], ib) and not lb[n:].any()


def test_birank_layout_sizes():
    """Bytes of each layout at one size: the paired layout halves the offset array of the 16-bit
    one, BiRank64 has none."""
    qr = require_gpu()
    n = 50 * 129024 + 5
    bits = datagen.bits(7, n, 0.5)
    d = to_dev(bits)
    announce("birank-layout-sizes")
    sizes = {L: qr.BiRank(d, n, layout=L).raw_layout() for L in (qr.QR_LAYOUT_16, qr.QR_LAYOUT_16P, qr.QR_LAYOUT_64,
                                                                  qr.QR_LAYOUT_16X2)}
    assert sizes[qr.QR_LAYOUT_16P][3] == (sizes[qr.QR_LAYOUT_16][3] + 1) // 2
    assert sizes[qr.QR_LAYOUT_64][3] == 0


# ------------------------------------------------------------------------------------------ QuadRank
# (name, bases per line, anchor data positions, lines per offset row, header slots)
QR_GEOM = {
    "16p": (480, (224,), 256, 32),
    "64": (384, (128,), None, 128),
    "24_8": (384, (64, 192, 320), 1 << 15, 128),
}


def qr_layout(qr, name):
    return {"16p": qr.QR_LAYOUT_16P, "64": qr.QR_LAYOUT_64, "24_8": qr.QR_LAYOUT_24_8}[name]


def qr_sizes(name):
    line, _, sb, _ = QR_GEOM[name]
    sizes = [0, 1, 31, 32, 33, 63, 64, 65, line - 1, line, line + 1, 128 * line - 1, 128 * line, 128 * line + 1,
             256 * line - 1, 256 * line, 256 * line + 1, 3 * 256 * line + 128 * line + 5, (1 << 20) + 3]
    if name == "24_8":
        sizes += [sb * line - 1, sb * line, sb * line + 1, 2 * sb * line + 12_345]
    return sizes


def qr_queries(name, n, seed, k=20000):
    line, anchors, sb, _ = QR_GEOM[name]
    parts = [datagen.queries(seed, n, k)]
    for a in anchors:
        parts.append(edge_queries(n, line, a, (sb or 256) * line))
    parts.append(edge_queries(n, line, anchors[0], 128 * line))         # pair middles and group starts
    if n <= 70000:
        parts.append(np.arange(n + 1, dtype=np.uint64))
    return np.unique(np.concatenate(parts))


def check_all_forms(qr, h, packed, n, q, c, tunes):
    want1 = oracle.rank_dna(packed, n, q, c)
    want4 = oracle.rank4_dna(packed, n, q)
    wantp = oracle.prefix_rank_dna(packed, n, q, c)
    dq, dc = to_dev(q), to_dev(c)
    for tune in tunes:
        h.set_tuning(**tune)
        assert np.array_equal(to_host_u64(h.rank(dq, dc)), want1), tune
        assert np.array_equal(to_host_u64(h.rank4(dq)).reshape(-1, 4), want4), tune
        assert np.array_equal(to_host_u64(h.prefix_rank(dq, dc)), wantp), tune


@pytest.mark.parametrize("name,n", [(nm, n) for nm in QR_GEOM for n in qr_sizes(nm)])
def test_quadrank_variant_edge_battery(name, n):
    qr = require_gpu()
    codes = qr_text(3000 + n, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=n + 2)
    q = qr_queries(name, n, 700 + n)
    c = datagen.symbols(800 + n, q.size)
    announce("quadrank-variant", name, n, q.size)
    h = qr.QuadRank(to_dev(packed), n, layout=qr_layout(qr, name))
    assert qr.lib().quadrank_layout_kind(h.h) == qr_layout(qr, name)
    check_all_forms(qr, h, packed, n, q, c, (dict(), dict(lanes=1), dict(lanes=2, per_lane=1, sweep=1024)))
    h.check()


@pytest.mark.parametrize("name", list(QR_GEOM))
@pytest.mark.parametrize("kind", ["allA", "allT", "periodic"])
def test_quadrank_variant_degenerate_texts(name, kind):
    qr = require_gpu()
    line = QR_GEOM[name][0]
    n = 3 * 256 * line + 999
    packed = datagen.pack2(qr_text(0, n, kind))
    q = qr_queries(name, n, 31)
    c = datagen.symbols(32, q.size)
    announce("quadrank-variant-degenerate", name, kind)
    h = qr.QuadRank(to_dev(packed), n, layout=qr_layout(qr, name))
    check_all_forms(qr, h, packed, n, q, c, (dict(),))


@pytest.mark.parametrize("name", list(QR_GEOM))
@pytest.mark.parametrize("tune", TUNINGS + SWEEP_TUNINGS)
def test_quadrank_variant_tunings(name, tune):
    qr = require_gpu()
    line = QR_GEOM[name][0]
    n = 2 * 256 * line + 4321
    packed = datagen.pack2(qr_text(177, n))
    q = np.concatenate([qr_queries(name, n, 178), datagen.queries(179, n, 100_003)])
    c = datagen.symbols(180, q.size)
    announce("quadrank-variant-tune", name, tune)
    h = qr.QuadRank(to_dev(packed), n, layout=qr_layout(qr, name))
    check_all_forms(qr, h, packed, n, q, c, (tune,))


@pytest.mark.parametrize("name", list(QR_GEOM))
def test_quadrank_variant_out_of_range(name):
    qr = require_gpu()
    n = 1000
    packed = datagen.pack2(datagen.dna_codes(5, n))
    q = np.array([0, n, n + 1, 3], dtype=np.uint64)
    c = np.array([0, 9, 1, 2], dtype=np.uint8)
    announce("quadrank-variant-out-of-range", name)
    h = qr.QuadRank(to_dev(packed), n, layout=qr_layout(qr, name))
    assert np.array_equal(to_host_u64(h.rank(to_dev(q), to_dev(c))), oracle.rank_dna(packed, n, q, c))
    with pytest.raises(qr.QRError):
        h.check()
    assert np.array_equal(to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4), oracle.rank4_dna(packed, n, q))
    with pytest.raises(qr.QRError):
        h.check()
    h.check()


def _padded_rank4(packed, n, pos):
    """rank4 at positions that may lie past n, over the text padded with A."""
    pos = np.asarray(pos, dtype=np.uint64)
    r = oracle.rank4_dna(packed, n, np.minimum(pos, n).astype(np.uint64))
    r[:, 0] += np.where(pos > n, pos - np.uint64(n), np.uint64(0))
    return r


def _planes(lines, first_slot):
    nl = lines.shape[0]
    lob = np.unpackbits(lines[:, 0::2].copy().view(np.uint8), bitorder="little").reshape(nl, 512)[:, first_slot:]
    hib = np.unpackbits(lines[:, 1::2].copy().view(np.uint8), bitorder="little").reshape(nl, 512)[:, first_slot:]
    return (lob + 2 * hib).reshape(-1)


def test_quadrank16p_structure_decoder():
    """Paired superblocks: s'_{i,c} = floor(rank(480 (256 i + 128), c) / 2^12); the four 16-bit
    deltas of line j minus BIAS = 128*480 - 224 for the lower 128 lines of a pair, plus 2^12 s',
    give rank4 at the line's middle (base 480 j + 224, over the A-padded text); bases round-trip."""
    qr = require_gpu()
    n = 5 * 122880 + 61440 + 4321
    codes = qr_text(556, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=4)
    announce("quadrank16p-structure", n)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_16P)
    lines, sup = h.export()
    nl = lines.shape[0]
    assert nl == n // 480 + 1 and sup.shape == ((nl - 1) // 256 + 1, 4) and sup.dtype == np.uint32
    i = np.arange(sup.shape[0], dtype=np.uint64)
    assert np.array_equal(sup.astype(np.uint64), _padded_rank4(packed, n, 480 * (256 * i + 128)) >> np.uint64(12))
    j = np.arange(nl, dtype=np.uint64)
    m16 = np.uint64(0xFFFF)
    w0, w1 = lines[:, 0], lines[:, 1]
    b = np.stack([w0 & m16, (w0 >> np.uint64(16)) & m16, w1 & m16, (w1 >> np.uint64(16)) & m16], axis=1).astype(np.int64)
    lower = ((j % np.uint64(256)) < np.uint64(128))[:, None]
    anchor = (sup[(j // np.uint64(256)).astype(np.int64)].astype(np.int64) << 12) + b - np.where(lower, 128 * 480 - 224, 0)
    assert np.array_equal(anchor.astype(np.uint64), _padded_rank4(packed, n, j * np.uint64(480) + np.uint64(224)))
    dec = _planes(lines, 32)
    assert np.array_equal(dec[:n], codes) and not dec[n:].any()


def test_quadrank64_structure_decoder():
    """QuadRank64: u64 words 0..3 of line j are rank(384 j + 128, A..T) (A-padded text); no offsets."""
    qr = require_gpu()
    n = 7 * 49152 + 4321
    codes = qr_text(557, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=5)
    announce("quadrank64-structure", n)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_64)
    lines, sup = h.export()
    nl = lines.shape[0]
    assert nl == n // 384 + 1 and sup.shape[0] == 0 and h.nbytes == nl * 128
    j = np.arange(nl, dtype=np.uint64)
    assert np.array_equal(lines[:, 0:4], _padded_rank4(packed, n, j * np.uint64(384) + np.uint64(128)))
    dec = _planes(lines, 128)
    assert np.array_equal(dec[:n], codes) and not dec[n:].any()


def test_quadrank24_8_structure_decoder():
    """QuadRank24_8: S_{i,c} = rank(384 * 2^15 i, c) exactly; per line and symbol, S + L1 is the rank
    at base 384 j + 64, + d1 at 384 j + 192, + d2 at 384 j + 320 (A-padded text); bases round-trip.
    Two superblocks of 2^15 lines are crossed."""
    qr = require_gpu()
    n = 2 * (1 << 15) * 384 + 9999
    codes = qr_text(558, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=6)
    announce("quadrank24_8-structure", n)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_24_8)
    lines, sup = h.export()
    nl = lines.shape[0]
    assert nl == n // 384 + 1 and sup.shape == ((nl - 1) // (1 << 15) + 1, 4) and sup.dtype == np.uint64
    i = np.arange(sup.shape[0], dtype=np.uint64)
    assert np.array_equal(sup, _padded_rank4(packed, n, i * np.uint64(384 << 15)))
    j = np.arange(nl, dtype=np.uint64)
    w = lines[:, 0:4].copy().view(np.uint32).reshape(nl, 8).astype(np.uint64)
    L1, d1, d2 = w[:, 0:4] & np.uint64(0xFFFFFF), w[:, 0:4] >> np.uint64(24), w[:, 4:8]
    assert (d2 <= 128).all() and (d1 <= 128).all()
    S = sup[(j >> np.uint64(15)).astype(np.int64)]
    base = j * np.uint64(384)
    assert np.array_equal(S + L1, _padded_rank4(packed, n, base + np.uint64(64)))
    assert np.array_equal(S + L1 + d1, _padded_rank4(packed, n, base + np.uint64(192)))
    assert np.array_equal(S + L1 + d1 + d2, _padded_rank4(packed, n, base + np.uint64(320)))
    dec = _planes(lines, 128)
    assert np.array_equal(dec[:n], codes) and not dec[n:].any()


def test_quadrank_layout_sizes():
    qr = require_gpu()
    n = 40 * 122880 + 5
    packed = datagen.pack2(datagen.dna_codes(8, n))
    d = to_dev(packed)
    announce("quadrank-layout-sizes")
    rows = {L: qr.QuadRank(d, n, layout=L).raw_layout()[3] for L in (qr.QR_LAYOUT_16, qr.QR_LAYOUT_16P, qr.QR_LAYOUT_64)}
    assert rows[qr.QR_LAYOUT_16P] == (rows[qr.QR_LAYOUT_16] + 1) // 2
    assert rows[qr.QR_LAYOUT_64] == 0


def test_layout_rejections():
    """Each structure refuses the other's variant and unknown layouts, on the host."""
    qr = require_gpu()
    announce("layout-rejections")
    bits = to_dev(datagen.bits(1, 1000))
    packed = to_dev(datagen.pack2(datagen.dna_codes(1, 1000)))
    for bad in (qr.QR_LAYOUT_24_8, 6, -1):
        with pytest.raises(qr.QRError):
            qr.BiRank(bits, 1000, layout=bad)
    for bad in (qr.QR_LAYOUT_16X2, 6, -1):
        with pytest.raises(qr.QRError):
            qr.QuadRank(packed, 1000, layout=bad)
