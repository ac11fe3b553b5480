"""Property tests (hypothesis, CPU): the oracle's rank, rank4, prefix_rank, count and locate
against brute force and their invariants on arbitrary small inputs, and the serving arena
allocator's invariants under arbitrary allocation/release sequences."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import datagen
import oracle
from paper_2602_04103_amd.serve import Arena

SETTINGS = settings(max_examples=60, deadline=None)
bits_st = st.lists(st.integers(0, 1), min_size=0, max_size=300)
dna_st = st.lists(st.integers(0, 3), min_size=0, max_size=200)


def pack_bits(bits):
    n = len(bits)
    words = np.zeros(max(1, (n + 63) // 64), np.uint64)
    for i, b in enumerate(bits):
        if b:
            words[i // 64] |= np.uint64(1) << np.uint64(i % 64)
    return words


@SETTINGS
@given(bits_st, st.integers(0, 2 ** 63))
def test_rank_bits_is_prefix_popcount(bits, garbage):
    n = len(bits)
    words = pack_bits(bits)
    if n % 64:  # bits past n must not matter
        words[-1] |= np.uint64(garbage) << np.uint64(n % 64)
    q = np.arange(n + 1, dtype=np.uint64)
    r = oracle.rank_bits(words, n, q)
    assert r.tolist() == [sum(bits[:k]) for k in range(n + 1)]


@SETTINGS
@given(dna_st)
def test_rank_rank4_prefix_rank_agree_with_brute_force(codes):
    c = np.array(codes, np.uint8)
    n = c.size
    packed = datagen.pack2(c, tail_garbage=True, seed=n)
    q = np.arange(n + 1, dtype=np.uint64)
    r4 = oracle.rank4_dna(packed, n, q)
    for s in range(4):
        want = [sum(1 for x in codes[:k] if x == s) for k in range(n + 1)]
        assert r4[:, s].tolist() == want
        assert oracle.rank_dna(packed, n, q, np.full(q.size, s, np.uint8)).tolist() == want
        pr = oracle.prefix_rank_dna(packed, n, q, np.full(q.size, s, np.uint8))
        assert pr.tolist() == [sum(1 for x in codes[:k] if x <= s) for k in range(n + 1)]
    assert np.array_equal(r4.sum(axis=1), q)


def brute_positions(text, p):
    t, m = list(text), len(p)
    return [i for i in range(len(t) + 1) if t[i:i + m] == list(p)] if m else list(range(len(t) + 1))


@SETTINGS
@given(st.lists(st.integers(0, 1), min_size=0, max_size=80),
       st.lists(st.lists(st.integers(0, 3), min_size=0, max_size=6), min_size=1, max_size=12))
def test_counts_and_locate_agree_with_brute_force(text01, pats):
    """Texts over {A, C} force many repeats; patterns over ACGT include absent symbols."""
    text = np.array(text01, np.uint8)
    n = text.size
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in pats])
    flat = np.array([x for p in pats for x in p], np.uint8)
    sa = oracle.suffix_array(text)
    b, _ = oracle.bwt(text, sa)
    want = [len(brute_positions(text01, p)) for p in pats]
    assert oracle.count_naive(text, flat, off).tolist() == want
    assert oracle.count_sa(text, sa, flat, off).tolist() == want
    assert oracle.count_backward(b, flat, off).tolist() == want
    start, pos = oracle.locate_sa(text, sa, flat, off)
    for i, p in enumerate(pats):
        got = pos[int(start[i]):int(start[i + 1])].tolist()
        assert sorted(got) == brute_positions(text01, p)
    assert sorted(sa.tolist()) == list(range(n + 1))


@SETTINGS
@given(st.lists(st.integers(0, 3), min_size=1, max_size=60),
       st.lists(st.lists(st.integers(0, 3), min_size=1, max_size=5), min_size=1, max_size=8))
def test_both_strands_is_the_sum_of_the_strands(text, pats):
    t = np.array(text, np.uint8)
    sa = oracle.suffix_array(t)
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in pats])
    flat = np.array([x for p in pats for x in p], np.uint8)
    rc = [oracle.revcomp(np.array(p, np.uint8)) for p in pats]
    assert all(np.array_equal(oracle.revcomp(r), np.array(p, np.uint8)) for r, p in zip(rc, pats))
    both = oracle.count_both_strands(t, sa, flat, off)
    want = [len(brute_positions(text, p)) + len(brute_positions(text, r.tolist())) for p, r in zip(pats, rc)]
    assert both.tolist() == want


@settings(max_examples=100, deadline=None)
@given(st.integers(1024, 1 << 20), st.lists(st.tuples(st.booleans(), st.integers(1, 50_000)), max_size=60))
def test_arena_blocks_never_overlap_and_bytes_balance(size, ops):
    a = Arena(size)
    live = []
    for is_alloc, nbytes in ops:
        if is_alloc or not live:
            at = a.alloc(nbytes)
            if at is not None:
                assert at % 256 == 0 and at + nbytes <= size
                for s0, n0 in live:
                    assert at + nbytes <= s0 or s0 + n0 <= at
                live.append((at, nbytes))
        else:
            s0, n0 = live.pop(len(live) // 2)
            a.release(s0, n0)
        # free ranges are sorted, disjoint and inside the arena
        for (x0, x1), (y0, y1) in zip(a.free, a.free[1:]):
            assert x1 < y0
        assert all(0 <= x0 < x1 <= size for x0, x1 in a.free)
        assert a.free_bytes + sum(n for _, n in live) == size
    for s0, n0 in live:
        a.release(s0, n0)
    assert a.free == [(0, size)]


# ------------------------------------------------------------------ serving scheduler (CPU stand-in)
_SERVE_TEXT = None


def _serve_text():
    global _SERVE_TEXT
    if _SERVE_TEXT is None:
        _SERVE_TEXT = datagen.dna_codes(5151, 3000)
    return _SERVE_TEXT


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 10_000), st.integers(1, 6), st.integers(8, 64), st.integers(0, 3), st.floats(1e3, 1e6),
       st.integers(1, 5))
def test_scheduler_serves_everything_within_limits(seed, slots, max_batch, budget_shift, rate, hold):
    """Arbitrary workloads, slot counts, batch caps and budgets (as small as a few requests): every
    request is served with the oracle's counts; in-flight batches never exceed the slots, reserved
    bytes never exceed the budget, nothing finishes before it arrives, and admission is FIFO."""
    from paper_2602_04103_amd.serve import Server, make_workload
    from tests.serve_fakes import FakeExecutor
    text = _serve_text()
    w = make_workload(seed, text, rate, duration_s=0.05, max_requests=30, max_size=48)
    one = max(w.batch_bytes(r, r + 1) for r in range(w.nreq))
    budget = one * (1 + budget_shift)
    polls = {}

    def ready(slot):  # a batch completes only after being polled `hold` times: overlap and reordering
        polls[slot] = polls.get(slot, 0) + 1
        if polls[slot] >= hold:
            polls[slot] = 0
            return True
        return False

    ex = FakeExecutor(w, lambda pat, off: oracle.count_naive(text, pat, off).astype(np.uint32), ready=ready)
    t = [0.0]

    def clock():
        t[0] += 1e-3
        return t[0]

    srv = Server(ex, slots=slots, budget_bytes=budget, max_batch_patterns=max_batch)
    res = srv.run(w, clock=clock, deadline_s=1e6)
    assert res.max_inflight <= slots and res.max_reserved_bytes <= budget
    assert np.all(res.finish_s >= w.arrival)
    for r in range(w.nreq):
        p0, p1 = int(w.req_off[r]), int(w.req_off[r + 1])
        want = oracle.count_naive(text, w.pat[int(w.off[p0]):int(w.off[p1])],
                                  (w.off[p0:p1 + 1] - w.off[p0]).astype(np.uint64)).astype(np.uint32)
        assert np.array_equal(srv.counts_of(w, r), want)
    starts = [r0 for _, r0, _, _ in ex.submitted]
    assert starts == sorted(starts) and starts[0] == 0          # batches cover the requests in order
    assert all(r1 == nxt for (_, _, r1, _), (_, nxt, _, _) in zip(ex.submitted, ex.submitted[1:]))
    assert ex.submitted[-1][2] == w.nreq
