"""CPU tests of the serving scheduler (continuous batching, slots, admission by device-memory
budget) with an oracle-backed stand-in executor: no GPU needed.  Failure handling is forced from
the host: slots that never finish, an injected free-memory value, a request larger than the budget."""
import numpy as np
import pytest

import datagen
import oracle
from paper_2602_04103_amd.serve import Arena, Server, Workload, make_workload
from tests.serve_fakes import FakeExecutor


def small_workload(seed=1, nreq=40, n=5000, rate=2e5):
    text = datagen.dna_codes(seed, n)
    w = make_workload(seed, text, rate, duration_s=1.0, max_requests=nreq, max_size=64)
    return text, w


def oracle_counter(text):
    return lambda pat, off: oracle.count_naive(text, pat, off).astype(np.uint32)


class StepClock:
    def __init__(self, dt=1e-3):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


def test_arena_alloc_release_any_order():
    a = Arena(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert x == 0 and y == 1024 and z == 2048
    assert a.alloc(2000) is None
    a.release(y, 1000)
    assert a.alloc(1000) == 1024
    a.release(x, 1000)
    a.release(z, 1000)
    a.release(1024, 1000)
    assert a.free == [(0, 4096)]
    assert a.alloc(4096) == 0


def test_results_match_oracle_per_request():
    text, w = small_workload()
    ex = FakeExecutor(w, oracle_counter(text))
    srv = Server(ex, slots=3, budget_bytes=1 << 20)
    st = srv.run(w, clock=StepClock())
    assert st.latency_s.size == w.nreq and np.all(st.latency_s >= 0)
    for r in range(w.nreq):
        p0, p1 = int(w.req_off[r]), int(w.req_off[r + 1])
        alone = oracle.count_naive(text, w.pat[int(w.off[p0]):int(w.off[p1])],
                                   (w.off[p0:p1 + 1] - w.off[p0]).astype(np.uint64))
        assert np.array_equal(srv.counts_of(w, r), alone.astype(np.uint32))


def test_slot_exhaustion_and_out_of_order_completion():
    text, w = small_workload(seed=2, nreq=60)
    polls = {}

    def ready(slot):  # higher slots finish first; every batch needs a few polls
        polls[slot] = polls.get(slot, 0) + 1
        return polls[slot] % (4 - slot) == 0

    ex = FakeExecutor(w, oracle_counter(text), ready=ready)
    srv = Server(ex, slots=3, budget_bytes=1 << 20, max_batch_patterns=50)
    st = srv.run(w, clock=StepClock(5e-3))
    assert st.max_inflight <= 3 and st.max_inflight >= 2
    assert not np.isnan(st.finish_s).any()
    # batches are contiguous FIFO ranges covering every request exactly once
    ranges = sorted((r0, r1) for _, r0, r1, _ in ex.submitted)
    assert ranges[0][0] == 0 and ranges[-1][1] == w.nreq
    assert all(a[1] == b[0] for a, b in zip(ranges, ranges[1:]))


def test_budget_limits_reserved_memory():
    text, w = small_workload(seed=3, nreq=50)
    one = max(w.batch_bytes(r, r + 1) for r in range(w.nreq))
    budget = 2 * one + 512
    ex = FakeExecutor(w, oracle_counter(text), ready=lambda s: np.random.rand() < 0.3)
    srv = Server(ex, slots=8, budget_bytes=budget)
    st = srv.run(w, clock=StepClock())
    assert st.max_reserved_bytes <= budget
    assert not np.isnan(st.finish_s).any()


def test_injected_free_memory_delays_admission():
    text, w = small_workload(seed=4, nreq=10)
    clock = StepClock()
    free = lambda: 0 if clock.t < 0.5 else 1 << 30   # no free device memory during the first 0.5 s
    ex = FakeExecutor(w, oracle_counter(text))
    srv = Server(ex, slots=2, budget_bytes=1 << 20, free_bytes_fn=free)
    st = srv.run(w, clock=clock)
    assert np.nanmin(st.finish_s) >= 0.5


def test_request_larger_than_budget_is_rejected():
    text, w = small_workload(seed=5, nreq=5)
    srv = Server(FakeExecutor(w, oracle_counter(text)), slots=1, budget_bytes=300)
    with pytest.raises(MemoryError):
        srv.run(w, clock=StepClock())


def test_stuck_executor_hits_deadline():
    text, w = small_workload(seed=6, nreq=5)
    srv = Server(FakeExecutor(w, oracle_counter(text), ready=lambda s: False), slots=1, budget_bytes=1 << 20)
    with pytest.raises(TimeoutError):
        srv.run(w, clock=StepClock(0.01), deadline_s=1.0)
