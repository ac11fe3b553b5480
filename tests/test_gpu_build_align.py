"""Builds from input that is 8-byte but not 16-byte aligned take the word-by-word load path of the
count and line passes instead of 16-byte loads: the structures must be byte-identical to builds
from aligned input, and their ranks must equal the oracle's."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu


def offset_view(words: np.ndarray) -> torch.Tensor:
    """A device copy of `words` starting 8 bytes into its allocation (8- but not 16-byte aligned)."""
    buf = torch.zeros(words.size + 1, dtype=torch.int64, device="cuda")
    buf[1:] = to_dev(words)
    v = buf[1:]
    assert v.data_ptr() % 16 == 8
    return v


@pytest.mark.parametrize("n", [1, 65_000, 3 * 64512 * 8 + 77, (1 << 22) + 5])
def test_birank_build_from_offset_input(n):
    qr = require_gpu()
    bits = datagen.bits(5000 + n, n, 0.4, tail_garbage=True)
    q = np.concatenate([datagen.queries(5001 + n, n, 50_000), np.array([0, n], np.uint64)])
    want = oracle.rank_bits(bits, n, q)
    for layout in (qr.QR_LAYOUT_16, qr.QR_LAYOUT_32):
        announce("birank-offset-build", n, layout)
        a = qr.BiRank(to_dev(bits), n, layout=layout)
        b = qr.BiRank(offset_view(bits), n, layout=layout)
        la, sa = a.export()
        lb, sb = b.export()
        assert np.array_equal(la, lb) and np.array_equal(sa, sb)
        assert np.array_equal(to_host_u64(b.rank(to_dev(q))), want)


@pytest.mark.parametrize("n", [1, 70_000, 2 * 61440 * 4 + 123, (1 << 22) + 9])
def test_quadrank_build_from_offset_input(n):
    qr = require_gpu()
    packed = datagen.pack2(datagen.dna_codes(6000 + n, n), tail_garbage=True, seed=n)
    q = np.concatenate([datagen.queries(6001 + n, n, 50_000), np.array([0, n], np.uint64)])
    c = datagen.symbols(6002 + n, q.size)
    want = oracle.rank_dna(packed, n, q, c)
    for layout in (qr.QR_LAYOUT_16, qr.QR_LAYOUT_32):
        announce("quadrank-offset-build", n, layout)
        a = qr.QuadRank(to_dev(packed), n, layout=layout)
        b = qr.QuadRank(offset_view(packed), n, layout=layout)
        la, sa = a.export()
        lb, sb = b.export()
        assert np.array_equal(la, lb) and np.array_equal(sa, sb)
        assert np.array_equal(to_host_u64(b.rank(to_dev(q), to_dev(c))), want)
