"""Randomised GPU parity (hypothesis, fixed seeds so every run draws the same cases): structures of
arbitrary size and density in both layouts, arbitrary query batches and every launch form, and
small FM-indexes over texts with repeats, each against the oracle."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import datagen
import oracle
from tests.gpu_util import require_gpu, to_dev, to_host_u64

pytestmark = pytest.mark.gpu

SETTINGS = settings(max_examples=25, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
TUNES = [dict(), dict(per_lane=2), dict(per_lane=4, grid_waves=4), dict(lanes=1, per_lane=2),
         dict(per_lane=1, sweep=1024), dict(per_lane=2, sweep=2048), dict(per_lane=1, sweep=4096)]


@SETTINGS
@given(st.one_of(st.integers(0, 3000), st.integers(50_000, 400_000)), st.floats(0.0, 1.0),
       st.one_of(st.integers(1, 300), st.integers(5_000, 30_000)), st.sampled_from(TUNES),
       st.booleans(), st.integers(0, 2 ** 31))
def test_birank_random(n, p, nq, tune, l32, s):
    qr = require_gpu()
    bits = datagen.bits(s, n, p, tail_garbage=True)
    q = datagen.queries(s + 1, n, nq)
    h = qr.BiRank(to_dev(bits), n, layout=qr.QR_LAYOUT_32 if l32 else qr.QR_LAYOUT_16)
    h.set_tuning(**tune)
    assert np.array_equal(to_host_u64(h.rank(to_dev(q))), oracle.rank_bits(bits, n, q))
    h.check()


@SETTINGS
@given(st.one_of(st.integers(0, 3000), st.integers(50_000, 300_000)),
       st.one_of(st.integers(1, 300), st.integers(5_000, 30_000)), st.sampled_from(TUNES), st.booleans(),
       st.integers(0, 2 ** 31))
def test_quadrank_random(n, nq, tune, l32, s):
    qr = require_gpu()
    codes = datagen.dna_codes(s, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=s)
    q = datagen.queries(s + 1, n, nq)
    c = datagen.symbols(s + 2, nq)
    h = qr.QuadRank(to_dev(packed), n, layout=qr.QR_LAYOUT_32 if l32 else qr.QR_LAYOUT_16)
    h.set_tuning(**tune)
    dq, dc = to_dev(q), to_dev(c)
    assert np.array_equal(to_host_u64(h.rank(dq, dc)), oracle.rank_dna(packed, n, q, c))
    assert np.array_equal(to_host_u64(h.rank4(dq)).reshape(-1, 4), oracle.rank4_dna(packed, n, q))
    assert np.array_equal(to_host_u64(h.prefix_rank(dq, dc)), oracle.prefix_rank_dna(packed, n, q, c))
    h.check()


@settings(max_examples=15, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(st.one_of(st.integers(1, 300), st.integers(3_000, 20_000)), st.integers(1, 600), st.integers(1, 9),
       st.sampled_from([1, 4, 8, 12]), st.sampled_from(["16", "16p", "32", "64", "24_8"]), st.integers(0, 63),
       st.integers(0, 2 ** 31))
def test_fm_random(n, npat, maxlen_div, kmer, layout, lead, s):
    """Any layout with one-lane queries; patterns also as 2-bit packed words, the stream starting
    `lead` filler bases before the first pattern (so patterns start anywhere inside a word)."""
    qr = require_gpu()
    text = datagen.dna_codes(s, n)
    if n > 2000:
        datagen.plant_repeats(s + 1, text, nseg=3, seglen=min(500, n // 4), copies=4, sub=0.01)
    maxlen = max(2, 250 // maxlen_div)
    pat, off, _ = datagen.patterns(s + 2, text, npat, minlen=1, maxlen=min(maxlen, max(1, n)))
    fm = qr.QuadFm.from_text(text, kmer=kmer, layout=qr.LAYOUT_BY_NAME[layout])
    sa = oracle.suffix_array(text)
    dp, do = to_dev(pat), to_dev(off)
    want = oracle.count_sa(text, sa, pat, off).astype(np.uint32)
    assert np.array_equal(fm.count(dp, do).cpu().numpy().view(np.uint32), want)
    assert np.array_equal(fm.count_batched(dp, do, 97).cpu().numpy().view(np.uint32), want)
    both = oracle.count_both_strands(text, sa, pat, off).astype(np.uint32)
    assert np.array_equal(fm.count(dp, do, both_strands=True).cpu().numpy().view(np.uint32), both)
    stream = np.concatenate([datagen.dna_codes(s + 3, lead), pat])
    p2, o2 = to_dev(datagen.pack2(stream)), to_dev(off + np.uint64(lead))
    got = fm.count_packed(p2, stream.size, o2).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    got = fm.count_packed(p2, stream.size, o2, both_strands=True).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, both)
    fm.check()
