"""GPU parity at the full scale configuration, in the launch settings the benchmark uses: BiRank on
2^36 bits (Bernoulli 0.5 and 0.05) and QuadRank on a 2^32-base text with planted repeats.  A full
2^24-query batch runs on the GPU and every output is compared with the oracle's; properties that
hold at any size are checked as well."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu

BATCH = 1 << 24
# the settings the tuner chooses on these structures (lane pairs with 2 queries per pair, in blocks
# of 128 or 256; the sweep form with tiles of 1024 or 4096) and a few neighbours; the last one also
# runs prefix_rank
BENCH_TUNINGS = [dict(lanes=2, per_lane=2, block=256, grid_waves=0), dict(lanes=2, per_lane=2, block=256, grid_waves=8),
                 dict(lanes=2, per_lane=8, block=256, grid_waves=8), dict(lanes=2, per_lane=2, block=256, sweep=1024),
                 dict(lanes=2, per_lane=2, block=128, grid_waves=0), dict(lanes=2, per_lane=1, block=256, sweep=4096),
                 dict(lanes=2, per_lane=1, block=256, sweep=1024)]


def boundary_queries(n, sb, line, mid):
    """Positions around every superblock start of a layout (and line middles next to it)."""
    pts = set()
    for k in range(1, n // sb + 1):
        for d in (-1, 0, 1, mid - 1, mid, mid + 1, line - 1, line, -line):
            pts.add(k * sb + d)
    return np.array(sorted(x for x in pts if 0 <= x <= n), dtype=np.uint64)


@pytest.mark.parametrize("p,seed", [(0.5, 3636), (0.05, 3637)])
def test_birank_2e36(p, seed):
    """Every layout the bench builds: the 16-bit one (superblocks of 64 lines), the 32-bit one
    (2^22-line superblocks, crossed 16 times at this size), paired superblocks, the 64-bit
    absolute lines and the quarter anchors."""
    qr = require_gpu()
    n = 1 << 36
    bits = datagen.bits(seed, n, p)
    total = int(np.unpackbits(bits.view(np.uint8)).sum(dtype=np.int64))
    q = datagen.queries(seed + 100, n, BATCH)
    fixed = np.concatenate([np.array([0, n, n - 1, 1 << 35], np.uint64), boundary_queries(n, (1 << 22) * 992, 992, 480),
                            boundary_queries(min(n, 64 * 64512 * 3), 64 * 1008, 1008, 496),
                            boundary_queries(min(n, 128 * 128 * 1008 * 3), 128 * 1008, 1008, 496),
                            boundary_queries(min(n, 64 * 960 * 3), 64 * 960, 960, 448),
                            boundary_queries(min(n, 64 * 63488 * 3), 64 * 992, 992, 224)])
    q[:fixed.size] = fixed
    dq = to_dev(q)
    want = oracle.rank_bits(bits, n, q)
    assert fixed.size < BATCH
    for layout in (qr.QR_LAYOUT_16, qr.QR_LAYOUT_32, qr.QR_LAYOUT_16P, qr.QR_LAYOUT_64, qr.QR_LAYOUT_16X2):
        announce("birank 2^36", p, "layout", layout)
        h = qr.BiRank(to_dev(bits), n, layout=layout)
        for tune in BENCH_TUNINGS:
            h.set_tuning(**tune)
            got = to_host_u64(h.rank(dq))
            assert np.array_equal(got, want), (layout, tune)
            assert got[1] == total and got[0] == 0
            assert np.all(got <= q)                              # at most q ones before q
        h.check()
        del h
        torch.cuda.empty_cache()


def test_quadrank_2e32_with_repeats():
    """Every layout the bench builds (rank, rank4 and prefix_rank): the 32-bit layout has its
    superblock boundary at 2^23 lines = 3758096384 bases, QuadRank24_8 one every 2^15 lines."""
    qr = require_gpu()
    n = 1 << 32
    codes = datagen.dna_codes(3202, n)
    datagen.plant_repeats(3203, codes, nseg=1000, seglen=10_000, copies=20, sub=0.01)
    hist = np.bincount(codes, minlength=4).astype(np.uint64)
    packed = datagen.pack2(codes)
    del codes
    q = datagen.queries(3204, n, BATCH)
    fixed = np.concatenate([np.array([n, 0], np.uint64), boundary_queries(n, (1 << 23) * 448, 448, 192),
                            boundary_queries(min(n, (1 << 15) * 384 * 4), (1 << 15) * 384, 384, 64),
                            boundary_queries(min(n, 256 * 480 * 4), 256 * 480, 480, 224)])
    q[:fixed.size] = fixed
    c = datagen.symbols(3205, BATCH)
    dq, dc = to_dev(q), to_dev(c)
    want1 = oracle.rank_dna(packed, n, q, c)
    want4 = oracle.rank4_dna(packed, n, q)
    wantp = oracle.prefix_rank_dna(packed, n, q, c)
    assert fixed.size < BATCH
    for layout in (qr.QR_LAYOUT_16, qr.QR_LAYOUT_32, qr.QR_LAYOUT_16P, qr.QR_LAYOUT_64, qr.QR_LAYOUT_24_8):
        announce("quadrank 2^32 layout", layout)
        h = qr.QuadRank(to_dev(packed), n, layout=layout)
        for tune in BENCH_TUNINGS:
            h.set_tuning(**tune)
            got1 = to_host_u64(h.rank(dq, dc))
            got4 = to_host_u64(h.rank4(dq)).reshape(-1, 4)
            assert np.array_equal(got1, want1), (layout, tune)
            assert np.array_equal(got4, want4), (layout, tune)
            assert np.array_equal(got4.sum(axis=1), q)           # sum over symbols = q
            assert np.array_equal(got4[0], hist)                 # rank4(n) = histogram
            assert np.array_equal(got1, got4[np.arange(BATCH), c.astype(np.int64)])
        # prefix_rank in the last tuning: the oracle's, and the partial sums of rank4
        gotp = to_host_u64(h.prefix_rank(dq, dc))
        assert np.array_equal(gotp, wantp), layout
        assert np.array_equal(gotp, np.cumsum(got4, axis=1)[np.arange(BATCH), c.astype(np.int64)])
        h.check()
        del h
        torch.cuda.empty_cache()
