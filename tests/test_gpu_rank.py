"""GPU parity: BiRank rank and QuadRank rank / rank4 against the oracle, bit-exact (integer
work: tolerance 0).  Covers the edge battery of sizes around line and superblock boundaries,
garbage tail bits, degenerate texts, every query-kernel tuning, out-of-range queries and a
structure decoder that checks every stored delta and superblock offset against the oracle."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import announce, edge_queries, require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu

BR_LINE, BR_MID, BR_SB = 1008, 496, 64512
QR_LINE, QR_MID, QR_SB = 480, 224, 61440

BR_SIZES = [0, 1, 63, 64, 65, 1007, 1008, 1009, 1504, 64511, 64512, 64513, 3 * 64512 + 1000, (1 << 20) + 17]
QR_SIZES = [0, 1, 31, 32, 33, 479, 480, 481, 704, 61439, 61440, 61441, 2 * 61440 + 5, (1 << 20) + 3]


def br_queries(n, seed, k=20000):
    q = np.concatenate([edge_queries(n, BR_LINE, BR_MID, BR_SB), datagen.queries(seed, n, k)])
    if n <= 70000:
        q = np.concatenate([q, np.arange(n + 1, dtype=np.uint64)])
    return q


def qr_queries(n, seed, k=20000):
    q = np.concatenate([edge_queries(n, QR_LINE, QR_MID, QR_SB), datagen.queries(seed, n, k)])
    if n <= 70000:
        q = np.concatenate([q, np.arange(n + 1, dtype=np.uint64)])
    return q


@pytest.mark.parametrize("p", [0.5, 0.05])
@pytest.mark.parametrize("n", BR_SIZES)
def test_birank_edge_battery(n, p):
    qr = require_gpu()
    bits = datagen.bits(17 + n, n, p, tail_garbage=True)
    q = br_queries(n, 5 + n)
    announce("birank", n, p, q.size)
    br = qr.BiRank(to_dev(bits), n)
    got = to_host_u64(br.rank(to_dev(q)))
    br.check()
    want = oracle.rank_bits(bits, n, q)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("fill", [0, 1])
def test_birank_constant_bitvectors(fill):
    qr = require_gpu()
    n = 5 * 64512 + 777
    bits = np.full((n + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF) if fill else np.uint64(0))
    q = br_queries(n, 3)
    announce("birank-constant", fill)
    got = to_host_u64(qr.BiRank(to_dev(bits), n).rank(to_dev(q)))
    assert np.array_equal(got, q if fill else np.zeros_like(q))


def test_birank_config0_full():
    """Bitvector of 2^24 iid Bernoulli(0.5) bits, 10^6 uniform queries in [0, n]."""
    qr = require_gpu()
    n = 1 << 24
    bits = datagen.bits(2024, n, 0.5)
    q = datagen.queries(2025, n, 10 ** 6)
    announce("birank-config0", n)
    got = to_host_u64(qr.BiRank(to_dev(bits), n).rank(to_dev(q)))
    assert np.array_equal(got, oracle.rank_bits(bits, n, q))


TUNINGS = [dict(per_lane=1), dict(per_lane=2), dict(per_lane=4), dict(per_lane=8), dict(block=64, per_lane=2),
           dict(per_lane=4, grid_waves=8), dict(per_lane=1, grid_waves=1), dict(lanes=1), dict(lanes=1, per_lane=4),
           dict(lanes=1, block=128, per_lane=2, grid_waves=4), dict(lanes=2, block=192, per_lane=8, grid_waves=2)]


@pytest.mark.parametrize("tune", TUNINGS)
def test_birank_tunings_agree(tune):
    qr = require_gpu()
    n = 3 * 64512 + 4321
    bits = datagen.bits(99, n, 0.5)
    q = np.concatenate([br_queries(n, 98), datagen.queries(97, n, 100_003)])
    announce("birank-tune", tune)
    br = qr.BiRank(to_dev(bits), n)
    br.set_tuning(**tune)
    got = to_host_u64(br.rank(to_dev(q)))
    assert np.array_equal(got, oracle.rank_bits(bits, n, q))


def test_birank_out_of_range():
    qr = require_gpu()
    n = 5000
    bits = datagen.bits(1, n)
    q = np.array([0, n, n + 1, 2 ** 63, 17], dtype=np.uint64)
    announce("birank-out-of-range")
    br = qr.BiRank(to_dev(bits), n)
    got = to_host_u64(br.rank(to_dev(q)))
    want = oracle.rank_bits(bits, n, q)
    assert np.array_equal(got, want)          # out-of-range entries are 2^64-1 on both sides
    with pytest.raises(qr.QRError) as ei:
        br.check()
    assert ei.value.status == qr.QR_ERANGE
    br.check()                                 # the sticky word was cleared


def test_birank_structure_decoder():
    """Every line's delta plus the shifted superblock offset equals the oracle rank at the line's
    middle; data bits round-trip; bounds b < 2^16, s < 2^32 hold by storage width."""
    qr = require_gpu()
    n = 7 * 64512 + 1234
    bits = datagen.bits(4242, n, 0.5, tail_garbage=True)
    announce("birank-structure", n)
    br = qr.BiRank(to_dev(bits), n)
    lines, sup = br.export()
    nl = lines.shape[0]
    assert nl == n // BR_LINE + 1 and sup.size == n // BR_SB + 1
    j = np.arange(nl, dtype=np.uint64)
    delta = (lines[:, 0] & np.uint64(0xFFFF)).astype(np.uint64)
    mids = np.minimum(j * BR_LINE + BR_MID, n).astype(np.uint64)   # past n the padded text has no more 1s
    want = oracle.rank_bits(bits, n, mids)
    got = (sup[(j // 64).astype(np.int64)].astype(np.uint64) << np.uint64(10)) + delta
    assert np.array_equal(got, want)
    # data round trip: line bits 16..1023 are input bits 1008 j ..
    lb = np.unpackbits(lines.view(np.uint8), bitorder="little").reshape(nl, 1024)[:, 16:].reshape(-1)
    ib = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    assert np.array_equal(lb[:n], ib)
    assert not lb[n:].any()


# ------------------------------------------------------------------------------------ QuadRank
def qr_text(seed, n, kind="uniform"):
    if kind == "uniform":
        codes = datagen.dna_codes(seed, n)
        if n >= 20000:
            datagen.plant_repeats(seed + 1, codes, nseg=5, seglen=2000, copies=4, sub=0.01)
    elif kind == "allA":
        codes = np.zeros(n, np.uint8)
    elif kind == "allT":
        codes = np.full(n, 3, np.uint8)
    else:  # periodic
        codes = (np.arange(n) % 7 % 4).astype(np.uint8)
    return codes


@pytest.mark.parametrize("n", QR_SIZES)
def test_quadrank_edge_battery(n):
    qr = require_gpu()
    codes = qr_text(300 + n, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=n)
    q = qr_queries(n, 7 + n)
    c = datagen.symbols(8 + n, q.size)
    announce("quadrank", n, q.size)
    h = qr.QuadRank(to_dev(packed), n)
    got1 = to_host_u64(h.rank(to_dev(q), to_dev(c)))
    got4 = to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4)
    h.check()
    assert np.array_equal(got1, oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(got4, oracle.rank4_dna(packed, n, q))


@pytest.mark.parametrize("kind", ["allA", "allT", "periodic"])
def test_quadrank_degenerate_texts(kind):
    qr = require_gpu()
    n = 3 * 61440 + 999
    codes = qr_text(0, n, kind)
    packed = datagen.pack2(codes)
    q = qr_queries(n, 31)
    c = datagen.symbols(32, q.size)
    announce("quadrank-degenerate", kind)
    h = qr.QuadRank(to_dev(packed), n)
    assert np.array_equal(to_host_u64(h.rank(to_dev(q), to_dev(c))), oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4), oracle.rank4_dna(packed, n, q))


def test_quadrank_config1_full():
    """Text of 2^28 iid bases; 10^7 rank(q, c) and 10^7 rank4(q) queries."""
    qr = require_gpu()
    n = 1 << 28
    codes = datagen.dna_codes(2028, n)
    packed = datagen.pack2(codes)
    del codes
    q1 = datagen.queries(2029, n, 10 ** 7)
    c1 = datagen.symbols(2030, 10 ** 7)
    q4 = datagen.queries(2031, n, 10 ** 7)
    announce("quadrank-config1", n)
    h = qr.QuadRank(to_dev(packed), n)
    got1 = to_host_u64(h.rank(to_dev(q1), to_dev(c1)))
    assert np.array_equal(got1, oracle.rank_dna(packed, n, q1, c1))
    got4 = to_host_u64(h.rank4(to_dev(q4))).reshape(-1, 4)
    assert np.array_equal(got4, oracle.rank4_dna(packed, n, q4))


@pytest.mark.parametrize("tune", TUNINGS)
def test_quadrank_tunings_agree(tune):
    qr = require_gpu()
    n = 2 * 61440 + 4321
    codes = qr_text(77, n)
    packed = datagen.pack2(codes)
    q = np.concatenate([qr_queries(n, 78), datagen.queries(79, n, 100_003)])
    c = datagen.symbols(80, q.size)
    announce("quadrank-tune", tune)
    h = qr.QuadRank(to_dev(packed), n)
    h.set_tuning(**tune)
    assert np.array_equal(to_host_u64(h.rank(to_dev(q), to_dev(c))), oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4), oracle.rank4_dna(packed, n, q))


def test_quadrank_out_of_range():
    qr = require_gpu()
    n = 1000
    packed = datagen.pack2(datagen.dna_codes(5, n))
    q = np.array([0, n, n + 1, 3], dtype=np.uint64)
    c = np.array([0, 9, 1, 2], dtype=np.uint8)
    announce("quadrank-out-of-range")
    h = qr.QuadRank(to_dev(packed), n)
    got = to_host_u64(h.rank(to_dev(q), to_dev(c)))
    assert np.array_equal(got, oracle.rank_dna(packed, n, q, c))
    with pytest.raises(qr.QRError):
        h.check()
    got4 = to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4)
    assert np.array_equal(got4, oracle.rank4_dna(packed, n, q))
    with pytest.raises(qr.QRError):
        h.check()
    h.check()


def test_quadrank_structure_decoder():
    qr = require_gpu()
    n = 5 * 61440 + 4321
    codes = qr_text(555, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=3)
    announce("quadrank-structure", n)
    h = qr.QuadRank(to_dev(packed), n)
    lines, sup = h.export()
    nl = lines.shape[0]
    assert nl == n // QR_LINE + 1 and sup.shape[0] == n // QR_SB + 1
    j = np.arange(nl, dtype=np.uint64)
    w0, w1 = lines[:, 0], lines[:, 1]
    deltas = np.stack([w0 & np.uint64(0xFFFF), (w0 >> np.uint64(16)) & np.uint64(0xFFFF),
                       w1 & np.uint64(0xFFFF), (w1 >> np.uint64(16)) & np.uint64(0xFFFF)], axis=1)
    mid = (j * QR_LINE + QR_MID).astype(np.uint64)
    # padded text: bases past n are A, so rank(mid, A) grows by mid - n there
    want = oracle.rank4_dna(packed, n, np.minimum(mid, n))
    want[:, 0] += np.where(mid > n, mid - np.uint64(n), np.uint64(0))
    got = (sup[(j // 128).astype(np.int64)].astype(np.uint64) << np.uint64(12)) + deltas
    assert np.array_equal(got, want)
    # data round trip through the transposed planes
    lo = lines[:, 0::2]
    hi = lines[:, 1::2]
    lob = np.unpackbits(lo.copy().view(np.uint8), bitorder="little").reshape(nl, 512)[:, 32:]
    hib = np.unpackbits(hi.copy().view(np.uint8), bitorder="little").reshape(nl, 512)[:, 32:]
    dec = (lob + 2 * hib).reshape(-1)
    assert np.array_equal(dec[:n], codes)
    assert not dec[n:].any()
