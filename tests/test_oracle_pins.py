"""Pins for the oracle: it is checked against things other than itself —
hand-worked examples, brute force in pure Python on tiny inputs, invariants
that the rank and count definitions imply, and library routines for special
cases.  Each pin is chosen so that a plausible slip in the oracle (an
off-by-one in q, a dropped partial word, a wrong sentinel order, a transposed
symbol code) fails at least one of them."""
import json
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def bits_to_words(s):
    n = len(s)
    w = np.zeros(max(1, (n + 63) // 64), dtype=np.uint64)
    for i, ch in enumerate(s):
        if ch == "1":
            w[i // 64] |= np.uint64(1 << (i % 64))
    return w


def codes_of(s):
    return np.array([CODE[ch] for ch in s], dtype=np.uint8)


def csr(pats):
    off = np.zeros(len(pats) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(p) for p in pats])
    flat = np.concatenate([codes_of(p) for p in pats]) if pats and off[-1] else np.zeros(0, np.uint8)
    return flat.astype(np.uint8), off


# ---------------------------------------------------------------- hand-worked examples
def test_golden_binary():
    g = json.load(open(GOLDEN))
    for e in g["binary"]:
        w = bits_to_words(e["bits"])
        got = oracle.rank_bits(w, len(e["bits"]), np.array(e["q"], dtype=np.uint64))
        assert got.tolist() == e["rank"]


def test_golden_dna():
    g = json.load(open(GOLDEN))
    for e in g["dna"]:
        codes = codes_of(e["text"])
        packed = datagen.pack2(codes)
        q = np.array(e["q"], dtype=np.uint64)
        assert oracle.rank4_dna(packed, codes.size, q).tolist() == e["rank4"]
        for c in range(4):
            got = oracle.rank_dna(packed, codes.size, q, np.full(q.size, c, np.uint8))
            assert got.tolist() == [r[c] for r in e["rank4"]]


def test_golden_fm_and_sa():
    g = json.load(open(GOLDEN))
    for e in g["fm"]:
        text = codes_of(e["text"])
        pat, off = csr(e["patterns"])
        sa = oracle.suffix_array(text)
        b, _ = oracle.bwt(text, sa)
        assert oracle.count_naive(text, pat, off).tolist() == e["count"]
        assert oracle.count_sa(text, sa, pat, off).tolist() == e["count"]
        assert oracle.count_backward(b, pat, off).tolist() == e["count"]
    for e in g["suffix_array"]:
        assert oracle.suffix_array(codes_of(e["text"])).tolist() == e["sa"]


# ---------------------------------------------------------------- binary rank
@pytest.mark.parametrize("n", [0, 1, 5, 63, 64, 65, 127, 128, 129, 300])
@pytest.mark.parametrize("p", [0.5, 0.05])
def test_rank_bits_bruteforce(n, p):
    w = datagen.bits(1000 + n, n, p, tail_garbage=True)
    bit = [(int(w[i // 64]) >> (i % 64)) & 1 for i in range(n)]
    q = np.arange(n + 1, dtype=np.uint64)
    got = oracle.rank_bits(w, n, q)
    want = [sum(bit[:k]) for k in range(n + 1)]
    assert got.tolist() == want


def test_rank_bits_invariants_and_special_cases():
    n = 200_003
    w = datagen.bits(7, n, 0.5, tail_garbage=True)
    t = np.unpackbits(w.view(np.uint8), bitorder="little")[:n].astype(np.uint64)
    q = np.arange(n + 1, dtype=np.uint64)
    r = oracle.rank_bits(w, n, q)
    assert r[0] == 0
    assert np.array_equal(r[1:] - r[:-1], t)          # rank(q+1) - rank(q) = t_q
    assert int(r[n]) == int(t.sum())                     # rank(n) = total popcount
    zeros = np.zeros_like(w)
    ones = np.full_like(w, np.uint64(0xFFFFFFFFFFFFFFFF))
    assert np.all(oracle.rank_bits(zeros, n, q) == 0)
    assert np.array_equal(oracle.rank_bits(ones, n, q), q)
    bad = oracle.rank_bits(w, n, np.array([n + 1, 2 ** 63], dtype=np.uint64))
    assert np.all(bad == oracle.BAD)


def test_rank_bits_large_values():
    # a multi-word input where ranks exceed 2^16 and positions cross many words
    n = (1 << 20) + 37
    ones = np.full((n + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF))
    q = datagen.queries(3, n, 1000)
    assert np.array_equal(oracle.rank_bits(ones, n, q), q)


# ---------------------------------------------------------------- DNA rank / rank4
@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 64, 100, 257])
def test_rank_dna_bruteforce(n):
    codes = datagen.dna_codes(11 + n, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=n)
    q = np.arange(n + 1, dtype=np.uint64)
    r4 = oracle.rank4_dna(packed, n, q)
    for c in range(4):
        want = [sum(1 for i in range(k) if codes[i] == c) for k in range(n + 1)]
        assert r4[:, c].tolist() == want
        got = oracle.rank_dna(packed, n, q, np.full(q.size, c, np.uint8))
        assert got.tolist() == want


def test_rank_dna_invariants():
    n = 100_001
    codes = datagen.dna_codes(5, n)
    datagen.plant_repeats(6, codes, nseg=20, seglen=500, copies=5, sub=0.01)
    packed = datagen.pack2(codes, tail_garbage=True, seed=1)
    q = np.arange(n + 1, dtype=np.uint64)
    r4 = oracle.rank4_dna(packed, n, q)
    assert np.array_equal(r4.sum(axis=1), q)                                   # sum_c rank(q,c) = q
    onehot = (codes[:, None] == np.arange(4)[None, :]).astype(np.uint64)
    assert np.array_equal(r4[1:] - r4[:-1], onehot)                            # rank(q+1,c)-rank(q,c) = [t_q=c]
    assert np.array_equal(r4[n], np.bincount(codes, minlength=4).astype(np.uint64))
    qs = datagen.queries(9, n, 5000)
    cs = datagen.symbols(10, 5000)
    r1 = oracle.rank_dna(packed, n, qs, cs)
    assert np.array_equal(r1, r4[qs.astype(np.int64), cs.astype(np.int64)])    # rank4 = 4 x rank1
    bad = oracle.rank_dna(packed, n, np.array([n + 1, 0], np.uint64), np.array([0, 4], np.uint8))
    assert np.all(bad == oracle.BAD)


def test_golden_prefix_rank():
    g = json.load(open(GOLDEN))
    for e in g["prefix_rank"]:
        codes = codes_of(e["text"])
        packed = datagen.pack2(codes, tail_garbage=True, seed=3)
        for c in range(4):
            q = np.array(e["q"], dtype=np.uint64)
            got = oracle.prefix_rank_dna(packed, codes.size, q, np.full(q.size, c, np.uint8))
            assert got.tolist() == [r[c] for r in e["prefix_rank"]]


@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 97])
def test_prefix_rank_bruteforce(n):
    codes = datagen.dna_codes(21 + n, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=n + 5)
    q = np.arange(n + 1, dtype=np.uint64)
    for c in range(4):
        want = [sum(1 for i in range(k) if codes[i] <= c) for k in range(n + 1)]
        assert oracle.prefix_rank_dna(packed, n, q, np.full(q.size, c, np.uint8)).tolist() == want


def test_prefix_rank_invariants():
    """prefix_rank(q, T) = q; at q = n the four values are the cumulative histogram; one step in q
    adds [t_q <= c]; out-of-range q or c give the error value."""
    n = 50_003
    codes = datagen.dna_codes(8, n)
    packed = datagen.pack2(codes, tail_garbage=True, seed=2)
    q = np.arange(n + 1, dtype=np.uint64)
    hist = np.cumsum(np.bincount(codes, minlength=4)).astype(np.uint64)
    for c in range(4):
        pr = oracle.prefix_rank_dna(packed, n, q, np.full(q.size, c, np.uint8))
        assert pr[n] == hist[c]
        assert np.array_equal(pr[1:] - pr[:-1], (codes <= c).astype(np.uint64))
        if c == 3:
            assert np.array_equal(pr, q)
    bad = oracle.prefix_rank_dna(packed, n, np.array([n + 1, 5], np.uint64), np.array([0, 4], np.uint8))
    assert np.all(bad == oracle.BAD)


def test_rank_dna_all_same_symbol():
    n = 4097
    for c in range(4):
        codes = np.full(n, c, np.uint8)
        packed = datagen.pack2(codes)
        q = np.arange(n + 1, dtype=np.uint64)
        r4 = oracle.rank4_dna(packed, n, q)
        for s in range(4):
            assert np.array_equal(r4[:, s], q if s == c else np.zeros_like(q))


# ---------------------------------------------------------------- FM count
def brute_count(text_s, p_s):
    if not p_s:
        return len(text_s) + 1
    return sum(1 for i in range(len(text_s) - len(p_s) + 1) if text_s[i:i + len(p_s)] == p_s)


def to_str(codes):
    return "".join("ACGT"[int(x)] for x in codes)


@pytest.mark.parametrize("seed", range(6))
def test_suffix_array_and_bwt_bruteforce(seed):
    n = [0, 1, 2, 17, 64, 300][seed]
    codes = datagen.dna_codes(seed, n)
    if seed % 2:
        codes[: n // 2] = 0  # long runs stress the '$' order
    s = to_str(codes) + "$"
    want = sorted(range(n + 1), key=lambda i: s[i:])     # '$' < 'A' < 'C' < 'G' < 'T' in ASCII
    sa = oracle.suffix_array(codes)
    assert sa.tolist() == want
    b, d = oracle.bwt(codes, sa)
    want_b = [("ACGT$".index(s[i - 1]) if i > 0 else 4) for i in want]
    assert b.tolist() == want_b
    assert d == want.index(0)


@pytest.mark.parametrize("text", ["", "A", "AA", "ACA", "GATT", "TTTTT", "ACGTA", "CACAC"])
def test_check_sa_accepts_exactly_the_sorted_order(text):
    """Over every permutation of the rows of a tiny T$, exactly one passes the checker: the order
    of sorting the suffixes of the string directly ('$' < A < C < G < T in ASCII)."""
    import itertools
    codes = codes_of(text)
    s = text + "$"
    want = sorted(range(len(s)), key=lambda i: s[i:])
    passing = [p for p in itertools.permutations(range(len(s))) if oracle.check_sa(codes, np.array(p)) == 0]
    assert passing == [tuple(want)]


@pytest.mark.parametrize("seed", range(5))
def test_check_sa_rejects_broken_arrays(seed):
    n = [50, 301, 1000, 4096, 20_000][seed]
    codes = datagen.dna_codes(900 + seed, n)
    if seed % 2:
        datagen.plant_repeats(950 + seed, codes, nseg=2, seglen=n // 10, copies=3, sub=0.01)
        codes[: n // 4] = 3                       # a long run: neighbours share long prefixes
    sa = oracle.suffix_array(codes)
    assert oracle.check_sa(codes, sa) == 0
    assert oracle.check_sa(codes, sa.astype(np.uint32)) == 0
    rng = np.random.default_rng(seed)
    k = int(rng.integers(0, n))
    swapped = sa.copy()
    swapped[[k, k + 1]] = swapped[[k + 1, k]]     # neighbouring rows exchanged
    assert oracle.check_sa(codes, swapped) == 2
    far = sa.copy()
    j = int(rng.integers(k + 2, n + 1)) if k + 2 <= n else 0
    far[[k, j]] = far[[j, k]]                       # two distant rows exchanged
    assert oracle.check_sa(codes, far) == 2
    dup = sa.copy()
    dup[k] = dup[(k + 7) % (n + 1)]                 # a value twice, so a row is missing
    assert oracle.check_sa(codes, dup) == 1
    out = sa.copy()
    out[k] = n + 1                                  # a value beyond the last row
    assert oracle.check_sa(codes, out) == 1
    assert oracle.check_sa(codes, sa[:-1]) == 1     # one row short
    neg = sa.copy()
    neg[k] = -1
    assert oracle.check_sa(codes, neg) == 1
    shifted = np.roll(sa, 1)                        # a permutation, but '$' no longer first
    assert oracle.check_sa(codes, shifted) == 2


@pytest.mark.parametrize("seed", range(4))
def test_count_three_ways_vs_bruteforce(seed):
    n = 400 + 37 * seed
    codes = datagen.dna_codes(100 + seed, n)
    datagen.plant_repeats(200 + seed, codes, nseg=3, seglen=40, copies=4, sub=0.02)
    pat, off, _ = datagen.patterns(300 + seed, codes, 300, minlen=1, maxlen=12, frac_sampled=0.7, sub=0.05)
    # edge patterns: empty, longer than the text, a code outside the alphabet
    extra = [np.zeros(0, np.uint8), datagen.dna_codes(5, n + 3), np.array([0, 7, 1], np.uint8)]
    flat = [pat[int(off[i]):int(off[i + 1])] for i in range(off.size - 1)] + extra
    off2 = np.zeros(len(flat) + 1, np.uint64)
    off2[1:] = np.cumsum([x.size for x in flat])
    pat2 = np.concatenate(flat).astype(np.uint8)
    ts = to_str(codes)
    want = []
    for x in flat:
        want.append(0 if np.any(x > 3) else brute_count(ts, to_str(x)))
    sa = oracle.suffix_array(codes)
    b, _ = oracle.bwt(codes, sa)
    assert oracle.count_naive(codes, pat2, off2).tolist() == want
    assert oracle.count_sa(codes, sa, pat2, off2).tolist() == want
    assert oracle.count_backward(b, pat2, off2).tolist() == want


def test_golden_locate():
    g = json.load(open(GOLDEN))
    for e in g["locate"]:
        text = codes_of(e["text"])
        pat, off = csr(e["patterns"])
        start, pos = oracle.locate_sa(text, oracle.suffix_array(text), pat, off)
        got = [pos[int(start[i]):int(start[i + 1])].tolist() for i in range(len(e["patterns"]))]
        assert got == e["positions"]


@pytest.mark.parametrize("seed", range(6))
def test_locate_bruteforce(seed):
    """Each pattern's positions are exactly the starts where it occurs (brute force), listed in
    increasing order of their suffixes (compared with the end of text smallest)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    text = datagen.dna_codes(700 + seed, n)
    if seed % 2:
        text[n // 2:] = text[: n - n // 2]  # a long repeat
    pats = [text[i:i + k] for i, k in zip(rng.integers(0, n, 40), rng.integers(1, 12, 40))]
    pats += [rng.integers(0, 4, k).astype(np.uint8) for k in rng.integers(1, 5, 20)]
    pats += [np.array([1, 5, 2], np.uint8), np.zeros(0, np.uint8)]
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in pats])
    flat = np.concatenate(pats).astype(np.uint8)
    start, pos = oracle.locate_sa(text, oracle.suffix_array(text), flat, off)
    s = "".join("ACGT"[c] for c in text)
    for i, p in enumerate(pats):
        got = pos[int(start[i]):int(start[i + 1])].tolist()
        if p.size and p.max() > 3:
            assert got == []
            continue
        ps = "".join("ACGT"[c] for c in p)
        occ = [k for k in range(n + 1) if s.startswith(ps, k)]
        assert sorted(got) == occ
        sufs = [s[k:] for k in got]
        assert sufs == sorted(sufs)                  # Python orders a proper prefix first, as '$' does


def test_count_extension_invariant():
    # sum over c of count(cP) = count(P) - [T starts with P]   (every occurrence but the one at 0 extends left)
    n = 5000
    codes = datagen.dna_codes(77, n)
    datagen.plant_repeats(78, codes, nseg=5, seglen=200, copies=6, sub=0.01)
    pats = [codes[i:i + L] for i, L in [(0, 3), (0, 6), (17, 4), (2000, 5), (4990, 10)]]
    pats += [datagen.dna_codes(900 + k, k) for k in range(1, 6)]
    sa = oracle.suffix_array(codes)
    b, _ = oracle.bwt(codes, sa)
    for P in pats:
        ext = [np.concatenate([[c], P]).astype(np.uint8) for c in range(4)]
        allp = [P.astype(np.uint8)] + ext
        off = np.zeros(6, np.uint64)
        off[1:] = np.cumsum([x.size for x in allp])
        cnt = oracle.count_backward(b, np.concatenate(allp), off)
        starts = int(np.array_equal(codes[:P.size], P))
        assert int(cnt[1:].sum()) == int(cnt[0]) - starts


def test_count_single_symbol_is_histogram():
    n = 3000
    codes = datagen.dna_codes(31, n)
    sa = oracle.suffix_array(codes)
    b, _ = oracle.bwt(codes, sa)
    pat = np.arange(4, dtype=np.uint8)
    off = np.arange(5, dtype=np.uint64)
    assert oracle.count_backward(b, pat, off).tolist() == np.bincount(codes, minlength=4).tolist()


def test_kmer_intervals_are_sa_ranges():
    n = 2000
    codes = datagen.dna_codes(41, n)
    datagen.plant_repeats(42, codes, nseg=4, seglen=100, copies=3, sub=0.01)
    sa = oracle.suffix_array(codes)
    b, _ = oracle.bwt(codes, sa)
    k = 4
    lo, hi = oracle.kmer_intervals(b, k)
    s = to_str(codes) + "$"
    prefixes = [s[i:i + k] for i in sa.tolist()]
    for w in range(4 ** k):
        kmer = "".join("ACGT"[(w >> (2 * (k - 1 - t))) & 3] for t in range(k))
        rows = [r for r, p in enumerate(prefixes) if p == kmer]
        if rows:
            assert (int(lo[w]), int(hi[w])) == (rows[0], rows[-1] + 1)
        else:
            assert int(hi[w]) <= int(lo[w])


# ---------------------------------------------------------------- generator determinism
def test_generators_deterministic():
    a = datagen.bits(5, 10_000, 0.05)
    b = datagen.bits(5, 10_000, 0.05)
    c = datagen.bits(6, 10_000, 0.05)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    dens = np.unpackbits(a.view(np.uint8)).mean()
    assert 0.04 < dens < 0.06
    t1 = datagen.dna_codes(9, 50_000)
    t2 = datagen.plant_repeats(3, t1.copy(), nseg=10, seglen=1000, copies=5, sub=0.01)
    t3 = datagen.plant_repeats(3, t1.copy(), nseg=10, seglen=1000, copies=5, sub=0.01)
    assert np.array_equal(t2, t3) and not np.array_equal(t1, t2)
    q = datagen.queries(1, 10, 100_000)
    assert q.max() == 10 and q.min() == 0                    # inclusive range [0, n]
    p1 = datagen.patterns(4, t2, 100)
    p2 = datagen.patterns(4, t2, 100)
    assert all(np.array_equal(x, y) for x, y in zip(p1, p2))
    L = np.diff(p1[1].astype(np.int64))
    assert L.min() >= 20 and L.max() <= 250


def test_revcomp_and_both_strands_by_hand():
    # ACGTTG reversed is GTTGCA, complemented CAACGT (worked by hand: A<->T, C<->G)
    assert "".join("ACGT"[c] for c in oracle.revcomp(codes_of("ACGTTG"))) == "CAACGT"
    text = codes_of("ACGTTGCAAT")
    sa = oracle.suffix_array(text)
    # "AT": forward once (positions 8-9); its reverse complement is AT again: 1 + 1 = 2
    # "TTG": forward once; reverse complement CAA occurs once (positions 6-8): 2
    # "GCA": forward once; reverse complement TGC occurs once (positions 4-6): 2
    # "ACG": forward once; reverse complement CGT occurs once (positions 1-3): 2
    # "TTT": 0 + reverse complement AAA: 0
    pat, off = csr(["AT", "TTG", "GCA", "ACG", "TTT", ""])
    assert oracle.count_both_strands(text, sa, pat, off).tolist() == [2, 2, 2, 2, 0, 11]
