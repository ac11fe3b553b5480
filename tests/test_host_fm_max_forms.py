"""The closed forms behind the largest-size FM test (the BWT of (ACGT)^k and its counts, both
strands included) checked against the oracle's suffix array, BWT and direct counts for small k."""
import numpy as np
import pytest

import datagen
import oracle
import tests.test_gpu_fm_max as T


@pytest.mark.parametrize("k", [1, 2, 5, 9, 33])
def test_closed_forms_match_the_oracle(k, monkeypatch):
    monkeypatch.setattr(T, "K", k)
    monkeypatch.setattr(T, "N", 4 * k)
    monkeypatch.setattr(T, "N1", 4 * k + 1)
    text = np.array([i % 4 for i in range(4 * k)], np.uint8)
    sa = oracle.suffix_array(text)
    b, dollar = oracle.bwt(text, sa)
    b = b.astype(np.uint8).copy()
    b[dollar] = 0  # '$' stored as A
    assert dollar == k
    assert np.array_equal(T.packed_bwt(), datagen.pack2(b))
    pats = [T.pattern(s, m) for s in range(4) for m in range(1, 4 * k + 3)] + [[0, 0], [3, 3], [], [0, 1, 3]]
    flat, off = T.csr(pats)
    assert oracle.count_naive(text, flat, off).tolist() == [T.expected(p) for p in pats]
    both = [T.expected(p) + T.expected(T.revcomp(p)) if p else T.N1 for p in pats]
    assert oracle.count_both_strands(text, sa, flat, off).tolist() == both
