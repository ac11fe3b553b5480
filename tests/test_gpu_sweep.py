"""GPU parity of the position-ordered (sweep) form of the rank kernels against the oracle,
bit-exact: BiRank rank and QuadRank rank / prefix_rank / rank4 in both inline layouts, every tile
size and 1 or 2 queries per lane pair, on query counts around the tile size (ragged last tiles),
queries that all fall in one bucket, already sorted or reversed queries, structures smaller than
the bucket count, and out-of-range queries and symbols (which must still raise the sticky error)."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu

SWEEPS = [dict(sweep=t, per_lane=p) for t in (1024, 2048, 4096) for p in (1, 2)]
COUNTS = [1, 255, 1023, 1024, 1025, 4095, 4096, 4097, 3 * 4096 + 17, 100_003]


def layouts(qr):
    return [qr.QR_LAYOUT_16, qr.QR_LAYOUT_32]


def query_sets(n, seed):
    """(name, queries) cases: uniform, one bucket, sorted, reversed, boundaries."""
    rng = np.random.default_rng(seed)
    u = datagen.queries(seed, n, 20_000)
    sets = [("uniform", u),
            ("one-position", np.full(5000, n // 2, np.uint64)),
            ("one-bucket", (n - rng.integers(0, min(n, max(1, n // 512)) + 1, 6000)).astype(np.uint64)),
            ("sorted", np.sort(u)),
            ("reversed", np.sort(u)[::-1].copy()),
            ("ends", np.array([0, n, 0, n] * 700, np.uint64))]
    return sets


@pytest.mark.parametrize("tune", SWEEPS)
@pytest.mark.parametrize("L", [0, 1])
def test_birank_sweep_counts(tune, L):
    qr = require_gpu()
    lay = layouts(qr)[L]
    n = 7 * 64512 + 1234
    bits = datagen.bits(700 + L, n, 0.5, tail_garbage=True)
    br = qr.BiRank(to_dev(bits), n, layout=lay)
    br.set_tuning(**tune)
    q_all = datagen.queries(701, n, max(COUNTS))
    want_all = oracle.rank_bits(bits, n, q_all)
    for nq in COUNTS:
        announce("birank-sweep", tune, L, nq)
        got = to_host_u64(br.rank(to_dev(q_all[:nq])))
        assert np.array_equal(got, want_all[:nq]), nq
    br.check()


@pytest.mark.parametrize("tune", SWEEPS)
@pytest.mark.parametrize("L", [0, 1])
def test_birank_sweep_query_shapes(tune, L):
    qr = require_gpu()
    lay = layouts(qr)[L]
    for n in (0, 1, 100, 255, 256, 257, 70_001, 3 * 64512 + 5):
        bits = datagen.bits(720 + n, n, 0.3, tail_garbage=True)
        br = qr.BiRank(to_dev(bits), n, layout=lay)
        br.set_tuning(**tune)
        for name, q in query_sets(n, 721 + n):
            announce("birank-sweep-shape", tune, L, n, name)
            got = to_host_u64(br.rank(to_dev(q)))
            assert np.array_equal(got, oracle.rank_bits(bits, n, q)), (n, name)
        br.check()


@pytest.mark.parametrize("L", [0, 1])
def test_birank_sweep_out_of_range(L):
    qr = require_gpu()
    n = 5000
    bits = datagen.bits(1, n)
    br = qr.BiRank(to_dev(bits), n, layout=layouts(qr)[L])
    br.set_tuning(sweep=1024)
    q = np.concatenate([datagen.queries(2, n, 3000), np.array([n + 1, 2 ** 63, 2 ** 64 - 1], np.uint64)])
    announce("birank-sweep-out-of-range", L)
    got = to_host_u64(br.rank(to_dev(q)))
    assert np.array_equal(got, oracle.rank_bits(bits, n, q))
    with pytest.raises(qr.QRError):
        br.check()
    br.check()  # the error word is cleared by the check that reports it


def qr_inputs(n, seed):
    codes = datagen.dna_codes(seed, n)
    if n >= 50_000:
        datagen.plant_repeats(seed + 1, codes, nseg=5, seglen=2000, copies=4, sub=0.01)
    return codes, datagen.pack2(codes, tail_garbage=True, seed=seed)


@pytest.mark.parametrize("tune", SWEEPS)
@pytest.mark.parametrize("L", [0, 1])
def test_quadrank_sweep_counts(tune, L):
    qr = require_gpu()
    n = 5 * 61440 + 321
    codes, packed = qr_inputs(n, 800 + L)
    h = qr.QuadRank(to_dev(packed), n, layout=layouts(qr)[L])
    h.set_tuning(**tune)
    q_all = datagen.queries(801, n, max(COUNTS))
    c_all = datagen.symbols(802, max(COUNTS))
    w_rank = oracle.rank_dna(packed, n, q_all, c_all)
    w_pre = oracle.prefix_rank_dna(packed, n, q_all, c_all)
    w_r4 = oracle.rank4_dna(packed, n, q_all)
    for nq in COUNTS:
        announce("quadrank-sweep", tune, L, nq)
        q, c = to_dev(q_all[:nq]), to_dev(c_all[:nq])
        assert np.array_equal(to_host_u64(h.rank(q, c)), w_rank[:nq]), nq
        assert np.array_equal(to_host_u64(h.prefix_rank(q, c)), w_pre[:nq]), nq
        assert np.array_equal(to_host_u64(h.rank4(q)).reshape(-1, 4), w_r4[:nq]), nq
    h.check()


@pytest.mark.parametrize("tune", SWEEPS)
@pytest.mark.parametrize("L", [0, 1])
def test_quadrank_sweep_query_shapes(tune, L):
    qr = require_gpu()
    for n in (0, 1, 100, 255, 256, 257, 61_441, 2 * 61440 + 7):
        codes, packed = qr_inputs(n, 820 + n)
        h = qr.QuadRank(to_dev(packed), n, layout=layouts(qr)[L])
        h.set_tuning(**tune)
        for name, q in query_sets(n, 821 + n):
            c = datagen.symbols(822 + n, q.size)
            announce("quadrank-sweep-shape", tune, L, n, name)
            qd, cd = to_dev(q), to_dev(c)
            assert np.array_equal(to_host_u64(h.rank(qd, cd)), oracle.rank_dna(packed, n, q, c)), (n, name)
            assert np.array_equal(to_host_u64(h.prefix_rank(qd, cd)), oracle.prefix_rank_dna(packed, n, q, c))
            assert np.array_equal(to_host_u64(h.rank4(qd)).reshape(-1, 4), oracle.rank4_dna(packed, n, q))
        h.check()


@pytest.mark.parametrize("tile", [1024, 2048])  # rank4: rows staged in LDS, then rows written one by one
@pytest.mark.parametrize("L", [0, 1])
def test_quadrank_sweep_out_of_range(L, tile):
    qr = require_gpu()
    n = 7000
    codes, packed = qr_inputs(n, 3)
    h = qr.QuadRank(to_dev(packed), n, layout=layouts(qr)[L])
    h.set_tuning(sweep=tile, per_lane=2)
    q = np.concatenate([datagen.queries(4, n, 3000), np.array([n + 1, 2 ** 63, 5], np.uint64)])
    c = datagen.symbols(5, q.size)
    announce("quadrank-sweep-bad-q", L)
    qd, cd = to_dev(q), to_dev(c)
    assert np.array_equal(to_host_u64(h.rank(qd, cd)), oracle.rank_dna(packed, n, q, c))
    with pytest.raises(qr.QRError):
        h.check()
    assert np.array_equal(to_host_u64(h.rank4(qd)).reshape(-1, 4), oracle.rank4_dna(packed, n, q))
    with pytest.raises(qr.QRError):
        h.check()
    c_bad = c.copy()
    c_bad[[0, 17, 2999]] = [4, 255, 7]
    q_ok = q[:3000]
    announce("quadrank-sweep-bad-c", L)
    got = to_host_u64(h.prefix_rank(to_dev(q_ok), to_dev(c_bad[:3000])))
    assert np.array_equal(got, oracle.prefix_rank_dna(packed, n, q_ok, c_bad[:3000]))
    with pytest.raises(qr.QRError):
        h.check()
    h.check()


def test_sweep_tuning_rejected():
    qr = require_gpu()
    n = 1000
    br = qr.BiRank(to_dev(datagen.bits(1, n)), n)
    h = qr.QuadRank(to_dev(datagen.pack2(datagen.dna_codes(2, n))), n)
    announce("sweep-tuning-rejected")
    for bad in (dict(sweep=512), dict(sweep=3000), dict(sweep=1024, lanes=1), dict(sweep=2048, per_lane=4)):
        for s in (br, h):
            with pytest.raises(qr.QRError):
                s.set_tuning(**bad)
    fm = qr.QuadFm.from_text(datagen.dna_codes(3, 500))
    with pytest.raises(qr.QRError):
        fm._tune(qr.lib().quadfm_set_tuning, sweep=1024)


@pytest.mark.parametrize("L", [0, 1])
def test_sweep_at_scale_sampled(L):
    """2^30 bits / 2^28 bases with 2^22 queries in the tile size and settings the tuner offers:
    every output checked against the oracle."""
    qr = require_gpu()
    nb = 1 << 30
    bits = datagen.bits(900 + L, nb, 0.5)
    q = datagen.queries(901, nb, 1 << 22)
    announce("birank-sweep-scale", L)
    br = qr.BiRank(to_dev(bits), nb, layout=layouts(qr)[L])
    want = oracle.rank_bits(bits, nb, q)
    for t in SWEEPS:
        br.set_tuning(**t)
        assert np.array_equal(to_host_u64(br.rank(to_dev(q))), want), t
    del br
    n = 1 << 28
    codes, packed = qr_inputs(n, 902 + L)
    c = datagen.symbols(903, q.size)
    q2 = datagen.queries(904, n, 1 << 22)
    announce("quadrank-sweep-scale", L)
    h = qr.QuadRank(to_dev(packed), n, layout=layouts(qr)[L])
    w1, w4 = oracle.rank_dna(packed, n, q2, c), oracle.rank4_dna(packed, n, q2)
    for t in (SWEEPS[1], SWEEPS[4]):
        h.set_tuning(**t)
        assert np.array_equal(to_host_u64(h.rank(to_dev(q2), to_dev(c))), w1), t
        assert np.array_equal(to_host_u64(h.rank4(to_dev(q2))).reshape(-1, 4), w4), t
