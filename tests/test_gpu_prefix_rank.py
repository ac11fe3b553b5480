"""GPU parity of prefix_rank(q, c) = #{i < q : t_i <= c} (the count of characters at most c, proposed
in the paper's closing section for a bidirectional FM-index) against the oracle, bit-exact
(tolerance 0), in both inline layouts: edge batteries around line, line-middle and build-group
boundaries with garbage tails, degenerate texts, every query-kernel tuning and out-of-range
inputs.  The full-scale case runs with the scale tests."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_util import announce, edge_queries, require_gpu, to_dev, to_host_u64
from tests.test_gpu_rank import TUNINGS, qr_text

pytestmark = pytest.mark.gpu

# (layout name, data bases per line, middle base, bases per build group of 128 lines)
GEOM = {16: (480, 224, 128 * 480), 32: (448, 192, 128 * 448)}
SIZES = [0, 1, 63, 64, 65, 223, 224, 225, 447, 448, 449, 479, 480, 481, 57345, 61441, 3 * 61440 + 77]


def layout_id(qr, L):
    return qr.QR_LAYOUT_16 if L == 16 else qr.QR_LAYOUT_32


def queries(n, seed, L, k=20000):
    line, mid, group = GEOM[L]
    q = np.concatenate([edge_queries(n, line, mid, group), datagen.queries(seed, n, k)])
    if n <= 70000:
        q = np.concatenate([q, np.arange(n + 1, dtype=np.uint64)])
    return q


@pytest.mark.parametrize("L", [16, 32])
@pytest.mark.parametrize("n", SIZES)
def test_prefix_rank_edge_battery(n, L):
    qr = require_gpu()
    codes = qr_text(1300 + n, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=n + 9)
    q = queries(n, 170 + n, L)
    c = datagen.symbols(180 + n, q.size)
    announce("prefix_rank", L, n, q.size)
    h = qr.QuadRank(to_dev(packed), n, layout=layout_id(qr, L))
    got = to_host_u64(h.prefix_rank(to_dev(q), to_dev(c)))
    h.check()
    assert np.array_equal(got, oracle.prefix_rank_dna(packed, n, q, c))


@pytest.mark.parametrize("L", [16, 32])
@pytest.mark.parametrize("kind", ["allA", "allT", "periodic"])
def test_prefix_rank_degenerate_texts(kind, L):
    qr = require_gpu()
    n = 2 * 61440 + 999
    packed = datagen.pack2(qr_text(0, n, kind))
    q = queries(n, 41, L)
    c = datagen.symbols(42, q.size)
    announce("prefix_rank-degenerate", L, kind)
    h = qr.QuadRank(to_dev(packed), n, layout=layout_id(qr, L))
    assert np.array_equal(to_host_u64(h.prefix_rank(to_dev(q), to_dev(c))), oracle.prefix_rank_dna(packed, n, q, c))


@pytest.mark.parametrize("L", [16, 32])
@pytest.mark.parametrize("tune", TUNINGS)
def test_prefix_rank_tunings_agree(tune, L):
    qr = require_gpu()
    n = 2 * 61440 + 4321
    packed = datagen.pack2(qr_text(277, n))
    q = np.concatenate([queries(n, 278, L), datagen.queries(279, n, 100_003)])
    c = datagen.symbols(280, q.size)
    announce("prefix_rank-tune", L, tune)
    h = qr.QuadRank(to_dev(packed), n, layout=layout_id(qr, L))
    h.set_tuning(**tune)
    assert np.array_equal(to_host_u64(h.prefix_rank(to_dev(q), to_dev(c))), oracle.prefix_rank_dna(packed, n, q, c))


@pytest.mark.parametrize("L", [16, 32])
def test_prefix_rank_out_of_range(L):
    qr = require_gpu()
    n = 1000
    packed = datagen.pack2(datagen.dna_codes(5, n))
    q = np.array([0, n, n + 1, 3, 2 ** 63], dtype=np.uint64)
    c = np.array([0, 3, 1, 4, 2], dtype=np.uint8)
    announce("prefix_rank-out-of-range", L)
    h = qr.QuadRank(to_dev(packed), n, layout=layout_id(qr, L))
    got = to_host_u64(h.prefix_rank(to_dev(q), to_dev(c)))
    assert np.array_equal(got, oracle.prefix_rank_dna(packed, n, q, c))
    assert got[1] == n                             # prefix_rank(n, T) = n
    with pytest.raises(qr.QRError):
        h.check()
    h.check()
