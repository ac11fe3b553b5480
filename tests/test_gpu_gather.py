"""GPU check of the random-line gather microbenchmark whose rates serve as the measured ceilings:
every launch form (1, 2, 4 or 8 lanes per line; plain, non-temporal line loads, non-temporal index
and result streams, both) returns for query i the 32-bit sum of the 32 words of line
floor(idx[i] * n_lines / 2^64), and the one-lane form the sum of the first 16 words for 64 bytes."""
import numpy as np
import pytest
import torch

from tests.gpu_util import announce, require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu


def expected(words, idx, n_lines, nwords):
    lines = ((idx.astype(object) * n_lines) >> 64).astype(np.int64)
    w = words.reshape(n_lines, 32)[:, :nwords].astype(np.uint64)
    return (w.sum(axis=1) & 0xFFFFFFFF)[lines].astype(np.uint64)


@pytest.mark.parametrize("nq", [1, 63, 1000, 70_001])
def test_gather_lanes_forms(nq):
    qr = require_gpu()
    rng = np.random.default_rng(nq)
    n_lines = 3001
    words = rng.integers(0, 2 ** 32, n_lines * 32, dtype=np.uint64).astype(np.uint32)
    idx = rng.integers(0, 2 ** 63, nq, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, nq, dtype=np.uint64)
    want = expected(words, idx, n_lines, 32)
    d_lines = to_dev(words.view(np.uint64))
    d_idx = to_dev(idx)
    for lanes in (1, 2, 4, 8):
        for flags in (0, qr.QR_GATHER_NONTEMPORAL, qr.QR_GATHER_STREAM_IO,
                      qr.QR_GATHER_NONTEMPORAL | qr.QR_GATHER_STREAM_IO):
            announce("gather-lanes", nq, lanes, flags)
            out = torch.full((nq,), -1, dtype=torch.int64, device="cuda")
            qr.qr_gather_lanes_bench(d_lines, n_lines, d_idx, lanes, out, flags=flags)
            assert np.array_equal(to_host_u64(out), want), (lanes, flags)
    for nbytes, nwords in ((64, 16), (128, 32)):
        announce("gather", nq, nbytes)
        out = torch.full((nq,), -1, dtype=torch.int64, device="cuda")
        qr.qr_gather_bench(d_lines, n_lines, d_idx, nbytes, out)
        assert np.array_equal(to_host_u64(out), expected(words, idx, n_lines, nwords)), nbytes
