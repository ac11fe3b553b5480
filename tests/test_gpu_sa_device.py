"""GPU parity of the device FM-index input preparation (suffix array of T$ by prefix doubling over a
radix sort, then the BWT and the locate sample) against the oracle's comparison-sort suffix array,
bit-exact: packed BWT words, the row of '$', the mark bits and the sampled SA values, on texts
around the sort's tile size (4096 suffixes), degenerate texts whose suffixes share very long
prefixes (many doubling steps), and texts with planted repeats.  Larger texts are compared with
the host SA-IS output, and the count test at 2^28 bases builds its index this way."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import datagen
import oracle
from tests.gpu_util import announce, require_gpu
from tests.test_gpu_fm import make_text

pytestmark = pytest.mark.gpu


def oracle_outputs(codes, rate):
    """Packed BWT words, '$' row, mark bits and samples computed from the oracle's suffix array."""
    n = codes.size
    sa = oracle.suffix_array(codes).astype(np.int64)
    b, dollar = oracle.bwt(codes, sa)
    b = b.astype(np.uint64)
    b[dollar] = 0  # '$' stored as A
    words = np.zeros(max(1, (n + 1 + 31) // 32), np.uint64)
    np.bitwise_or.at(words, np.arange(n + 1) // 32, b << (2 * (np.arange(n + 1) % 32)).astype(np.uint64))
    marks = samples = None
    if rate:
        m = (sa % rate == 0)
        bits = np.zeros(max(1, (n + 1 + 63) // 64) * 64, np.uint8)
        bits[:n + 1] = m
        marks = np.packbits(bits, bitorder="little").view(np.uint64)
        samples = sa[m].astype(np.uint32)
    return words, dollar, marks, samples


def device_outputs(qr, codes, rate, with_sa=False):
    t = torch.from_numpy(np.ascontiguousarray(codes)).cuda()
    sa = torch.empty(codes.size + 1, dtype=torch.int32, device="cuda") if with_sa else None
    bwt, dollar, marks, samples = qr.quadfm_index_device(t, rate, sa=sa)
    out = [bwt.cpu().numpy().view(np.uint64), dollar]
    out += [marks.cpu().numpy().view(np.uint64), samples.cpu().numpy().view(np.uint32)] if rate else [None, None]
    out.append(sa.cpu().numpy().view(np.uint32) if with_sa else None)
    return out


def check_against_oracle(qr, codes, rate):
    got = device_outputs(qr, codes, rate, with_sa=rate > 0)
    want = oracle_outputs(codes, rate)
    assert got[1] == want[1]
    assert np.array_equal(got[0], want[0])
    if rate:
        assert np.array_equal(got[2], want[2]) and np.array_equal(got[3], want[3])
        # the suffix array handed out is the oracle's (and passes the oracle's direct check)
        assert np.array_equal(got[4].astype(np.int64), oracle.suffix_array(codes))
        assert oracle.check_sa(codes, got[4]) == 0


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 20, 21, 22, 31, 32, 33, 100, 1000, 4094, 4095, 4096, 4097, 8191,
                               20_000, 65_537])
def test_device_sa_random_texts(n):
    qr = require_gpu()
    codes = datagen.dna_codes(900 + n, n)
    announce("device-sa", n)
    check_against_oracle(qr, codes, 0)
    check_against_oracle(qr, codes, 7 if n > 7 else 1)


def fibonacci_word(n):
    """The Fibonacci word over {A, C} (s_k = s_{k-1} s_{k-2}), cut to n characters."""
    a, b = [0], [0, 1]
    while len(b) < n:
        a, b = b, b + a
    return np.array(b[:n], np.uint8)


def mixed_repeats(n):
    """Random text with copies of segments of 30, 300, 3000 and 9000 characters, so that groups of
    suffixes finish in different doubling steps."""
    codes = datagen.dna_codes(12, n)
    at = 0
    for k, length in enumerate((30, 300, 3000, 9000)):
        seg = datagen.dna_codes(13 + k, length)
        for _ in range(2 if length > 1000 else 5):
            codes[at:at + length] = seg
            at += length + 7
    return codes


@pytest.mark.parametrize("kind", ["allA", "allT", "period7", "tiled37", "halves", "fibonacci", "mixed"])
def test_device_sa_degenerate_texts(kind):
    """Suffixes sharing prefixes of thousands of characters: many doubling steps; groups that
    finish in different steps (only unfinished groups are sorted again)."""
    qr = require_gpu()
    n = 30_001
    if kind == "allA":
        codes = np.zeros(n, np.uint8)
    elif kind == "allT":
        codes = np.full(n, 3, np.uint8)
    elif kind == "period7":
        codes = (np.arange(n) % 7 % 4).astype(np.uint8)
    elif kind == "tiled37":
        codes = np.tile(datagen.dna_codes(9, 37), n // 37 + 1)[:n].copy()
    elif kind == "fibonacci":
        codes = fibonacci_word(n)
    elif kind == "mixed":
        codes = mixed_repeats(n)
    else:
        h = datagen.dna_codes(10, n // 2)
        codes = np.concatenate([h, h, datagen.dna_codes(11, n - 2 * h.size)])
    announce("device-sa-degenerate", kind)
    check_against_oracle(qr, codes, 0)
    check_against_oracle(qr, codes, 32)


@pytest.mark.parametrize("rate", [1, 32, 5000])
def test_device_sa_repeats_1m(rate):
    """2^20 bases with planted repeats (10-kb segments x 20 copies, 1% substitutions)."""
    qr = require_gpu()
    n = 1 << 20
    codes = make_text(33, n)
    announce("device-sa-repeats", n, rate)
    check_against_oracle(qr, codes, rate)
    a, b = device_outputs(qr, codes, rate), device_outputs(qr, codes, rate)   # deterministic
    assert a[1] == b[1] and all(np.array_equal(x, y) for x, y in zip(a[0:1] + a[2:], b[0:1] + b[2:]))


def test_device_sa_matches_host_at_2e24():
    qr = require_gpu()
    n = (1 << 24) + 12345
    codes = datagen.dna_codes(2424, n)
    datagen.plant_repeats(2425, codes, nseg=100, seglen=10_000, copies=20, sub=0.01)
    announce("device-sa-vs-host", n)
    got = device_outputs(qr, codes, 32)
    bwt, dollar, marks, samples = qr.quadfm_index_host(codes, 32)
    assert got[1] == dollar
    assert np.array_equal(got[0], bwt) and np.array_equal(got[2], marks) and np.array_equal(got[3], samples)


def test_device_sa_rejects_bad_codes():
    qr = require_gpu()
    announce("device-sa-bad")
    t = torch.from_numpy(np.array([0, 1, 4, 2], np.uint8)).cuda()
    with pytest.raises(qr.QRError):
        qr.quadfm_index_device(t, 0)


@settings(max_examples=30, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(st.integers(0, 6000), st.sampled_from(["random", "periodic", "repeats", "runs"]), st.integers(1, 60),
       st.sampled_from([0, 1, 3, 32]), st.integers(0, 2 ** 31))
def test_device_sa_random_structures(n, kind, period, rate, seed):
    """Randomised texts (hypothesis, derandomised): uniform, periodic with a random period, random
    segments copied with substitutions, and long single-symbol runs, so groups of suffixes finish
    after any number of doubling steps."""
    qr = require_gpu()
    rng = np.random.default_rng(seed)
    if kind == "random":
        codes = rng.integers(0, 4, n, dtype=np.uint8)
    elif kind == "periodic":
        codes = np.tile(rng.integers(0, 4, period, dtype=np.uint8), n // period + 1)[:n].copy()
    elif kind == "repeats":
        codes = rng.integers(0, 4, n, dtype=np.uint8)
        seg = rng.integers(0, 4, max(1, n // 8), dtype=np.uint8)
        for _ in range(4):
            at = int(rng.integers(0, max(1, n - seg.size + 1)))
            copy = seg.copy()
            flip = rng.random(seg.size) < 0.01
            copy[flip] = (copy[flip] + 1) % 4
            codes[at:at + seg.size] = copy[:max(0, min(seg.size, n - at))]
    else:
        codes = np.repeat(rng.integers(0, 4, max(1, n // max(1, period * 20) + 1), dtype=np.uint8),
                          period * 20)[:n].copy()
    announce("device-sa-random", n, kind, period, rate, seed)
    check_against_oracle(qr, codes, rate)
