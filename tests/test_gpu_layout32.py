"""GPU parity of the 32-bit inline layouts (BiRank32 and QuadRank32 of Sections 3 and 4) against the
oracle, bit-exact (tolerance 0): edge batteries around line, line-middle and build-group
boundaries, garbage tail bits, degenerate inputs, every query-kernel tuning, out-of-range queries,
and structure decoders that check every stored 32-bit delta and exact 64-bit offset.  Superblock
boundaries of these layouts (2^22 and 2^23 lines) are crossed by the full-scale tests."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import announce, edge_queries, require_gpu, to_dev, to_host_u64
from tests.test_gpu_rank import TUNINGS, qr_text

pytestmark = pytest.mark.gpu

BR_LINE, BR_MID, BR_GROUP = 992, 480, 64 * 992
QR_LINE, QR_MID, QR_GROUP = 448, 192, 128 * 448

BR_SIZES = [0, 1, 31, 32, 33, 479, 480, 481, 991, 992, 993, 1472, 63487, 63488, 63489, 3 * 63488 + 1000,
            (1 << 20) + 17]
QR_SIZES = [0, 1, 63, 64, 65, 191, 192, 193, 447, 448, 449, 640, 57343, 57344, 57345, 2 * 57344 + 5, (1 << 20) + 3]


def queries(n, seed, line, mid, group, k=20000):
    q = np.concatenate([edge_queries(n, line, mid, group), datagen.queries(seed, n, k)])
    if n <= 70000:
        q = np.concatenate([q, np.arange(n + 1, dtype=np.uint64)])
    return q


@pytest.mark.parametrize("p", [0.5, 0.05])
@pytest.mark.parametrize("n", BR_SIZES)
def test_birank32_edge_battery(n, p):
    qr = require_gpu()
    bits = datagen.bits(170 + n, n, p, tail_garbage=True)
    q = queries(n, 50 + n, BR_LINE, BR_MID, BR_GROUP)
    announce("birank32", n, p, q.size)
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_32)
    assert qr.lib().birank_layout_kind(br.h) == qr.QR_LAYOUT_32
    got = to_host_u64(br.rank(to_dev(q)))
    br.check()
    assert np.array_equal(got, oracle.rank_bits(bits, n, q))


@pytest.mark.parametrize("fill", [0, 1])
def test_birank32_constant_bitvectors(fill):
    qr = require_gpu()
    n = 5 * 63488 + 777
    bits = np.full((n + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF) if fill else np.uint64(0))
    q = queries(n, 3, BR_LINE, BR_MID, BR_GROUP)
    announce("birank32-constant", fill)
    got = to_host_u64(qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_32).rank(to_dev(q)))
    assert np.array_equal(got, q if fill else np.zeros_like(q))


@pytest.mark.parametrize("tune", TUNINGS)
def test_birank32_tunings_agree(tune):
    qr = require_gpu()
    n = 3 * 63488 + 4321
    bits = datagen.bits(199, n, 0.5)
    q = np.concatenate([queries(n, 198, BR_LINE, BR_MID, BR_GROUP), datagen.queries(197, n, 100_003)])
    announce("birank32-tune", tune)
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_32)
    br.set_tuning(**tune)
    assert np.array_equal(to_host_u64(br.rank(to_dev(q))), oracle.rank_bits(bits, n, q))


def test_birank32_out_of_range():
    qr = require_gpu()
    n = 5000
    bits = datagen.bits(1, n)
    q = np.array([0, n, n + 1, 2 ** 63, 17], dtype=np.uint64)
    announce("birank32-out-of-range")
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_32)
    assert np.array_equal(to_host_u64(br.rank(to_dev(q))), oracle.rank_bits(bits, n, q))
    with pytest.raises(qr.QRError):
        br.check()
    br.check()


def test_birank32_structure_decoder():
    """b_j + s_{j / 2^22} equals the oracle rank at line j's middle (bit 992 j + 480), and the data
    bits round-trip."""
    qr = require_gpu()
    n = 7 * 63488 + 1234
    bits = datagen.bits(4343, n, 0.5, tail_garbage=True)
    announce("birank32-structure", n)
    br = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_32)
    lines, sup = br.export()
    nl = lines.shape[0]
    assert nl == n // BR_LINE + 1 and sup.size == 1 and sup.dtype == np.uint64 and sup[0] == 0
    j = np.arange(nl, dtype=np.uint64)
    delta = lines[:, 0] & np.uint64(0xFFFFFFFF)
    want = oracle.rank_bits(bits, n, np.minimum(j * BR_LINE + BR_MID, n).astype(np.uint64))
    assert np.array_equal(sup[(j >> np.uint64(22)).astype(np.int64)] + delta, want)
    lb = np.unpackbits(lines.view(np.uint8), bitorder="little").reshape(nl, 1024)[:, 32:].reshape(-1)
    ib = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    assert np.array_equal(lb[:n], ib)
    assert not lb[n:].any()


@pytest.mark.parametrize("n", QR_SIZES)
def test_quadrank32_edge_battery(n):
    qr = require_gpu()
    codes = qr_text(900 + n, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=n + 1)
    q = queries(n, 70 + n, QR_LINE, QR_MID, QR_GROUP)
    c = datagen.symbols(80 + n, q.size)
    announce("quadrank32", n, q.size)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32)
    assert qr.lib().quadrank_layout_kind(h.h) == qr.QR_LAYOUT_32
    got1 = to_host_u64(h.rank(to_dev(q), to_dev(c)))
    got4 = to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4)
    h.check()
    assert np.array_equal(got1, oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(got4, oracle.rank4_dna(packed, n, q))


@pytest.mark.parametrize("kind", ["allA", "allT", "periodic"])
def test_quadrank32_degenerate_texts(kind):
    qr = require_gpu()
    n = 3 * 57344 + 999
    packed = datagen.pack2(qr_text(0, n, kind))
    q = queries(n, 31, QR_LINE, QR_MID, QR_GROUP)
    c = datagen.symbols(32, q.size)
    announce("quadrank32-degenerate", kind)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32)
    assert np.array_equal(to_host_u64(h.rank(to_dev(q), to_dev(c))), oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4), oracle.rank4_dna(packed, n, q))


@pytest.mark.parametrize("tune", TUNINGS)
def test_quadrank32_tunings_agree(tune):
    qr = require_gpu()
    n = 2 * 57344 + 4321
    packed = datagen.pack2(qr_text(177, n))
    q = np.concatenate([queries(n, 178, QR_LINE, QR_MID, QR_GROUP), datagen.queries(179, n, 100_003)])
    c = datagen.symbols(180, q.size)
    announce("quadrank32-tune", tune)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32)
    h.set_tuning(**tune)
    assert np.array_equal(to_host_u64(h.rank(to_dev(q), to_dev(c))), oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4), oracle.rank4_dna(packed, n, q))


def test_quadrank32_out_of_range():
    qr = require_gpu()
    n = 1000
    packed = datagen.pack2(datagen.dna_codes(5, n))
    q = np.array([0, n, n + 1, 3], dtype=np.uint64)
    c = np.array([0, 9, 1, 2], dtype=np.uint8)
    announce("quadrank32-out-of-range")
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32)
    assert np.array_equal(to_host_u64(h.rank(to_dev(q), to_dev(c))), oracle.rank_dna(packed, n, q, c))
    with pytest.raises(qr.QRError):
        h.check()
    assert np.array_equal(to_host_u64(h.rank4(to_dev(q))).reshape(-1, 4), oracle.rank4_dna(packed, n, q))
    with pytest.raises(qr.QRError):
        h.check()
    h.check()


def test_quadrank32_structure_decoder():
    """Four 32-bit deltas in pair 0 (lo_0 = b_A | b_C << 32, hi_0 = b_G | b_T << 32) plus the exact
    offsets give the oracle rank4 at each line's middle (base 448 j + 192) over the A-padded text,
    and the transposed planes round-trip the bases."""
    qr = require_gpu()
    n = 5 * 57344 + 4321
    codes = qr_text(556, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=4)
    announce("quadrank32-structure", n)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32)
    lines, sup = h.export()
    nl = lines.shape[0]
    assert nl == n // QR_LINE + 1 and sup.shape == (1, 4) and sup.dtype == np.uint64 and not sup.any()
    j = np.arange(nl, dtype=np.uint64)
    m32 = np.uint64(0xFFFFFFFF)
    w0, w1 = lines[:, 0], lines[:, 1]
    deltas = np.stack([w0 & m32, w0 >> np.uint64(32), w1 & m32, w1 >> np.uint64(32)], axis=1)
    mid = (j * QR_LINE + QR_MID).astype(np.uint64)
    want = oracle.rank4_dna(packed, n, np.minimum(mid, n))
    want[:, 0] += np.where(mid > n, mid - np.uint64(n), np.uint64(0))
    assert np.array_equal(sup[(j >> np.uint64(23)).astype(np.int64)] + deltas, want)
    lob = np.unpackbits(lines[:, 0::2].copy().view(np.uint8), bitorder="little").reshape(nl, 512)[:, 64:]
    hib = np.unpackbits(lines[:, 1::2].copy().view(np.uint8), bitorder="little").reshape(nl, 512)[:, 64:]
    dec = (lob + 2 * hib).reshape(-1)
    assert np.array_equal(dec[:n], codes)
    assert not dec[n:].any()
