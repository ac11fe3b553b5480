"""Test double for the serving scheduler: an executor that counts on the CPU and completes batches
when the test says so (to force out-of-order completion)."""
from typing import Callable, List, Optional

import numpy as np

from paper_2602_04103_amd.serve import Workload


class FakeExecutor:
    """CPU stand-in: counts with `count_fn(pat, off)` and completes a batch once `ready(slot)` says so
    (tests use it to force out-of-order completion)."""

    def __init__(self, workload: Workload, count_fn: Callable, ready: Optional[Callable] = None):
        self.w, self.count_fn = workload, count_fn
        self.ready = ready or (lambda slot: True)
        self.cnt = np.zeros(int(workload.off.size - 1), dtype=np.uint32)
        self.submitted: List[tuple] = []

    def submit(self, slot: int, r0: int, r1: int, base: int):
        w = self.w
        p0, p1 = int(w.req_off[r0]), int(w.req_off[r1])
        off = (w.off[p0:p1 + 1] - w.off[p0]).astype(np.uint64)
        self.cnt[p0:p1] = self.count_fn(w.pat[int(w.off[p0]):int(w.off[p1])], off)
        self.submitted.append((slot, r0, r1, base))

    def poll(self, slot: int) -> bool:
        return bool(self.ready(slot))

    def counts(self, p0: int, p1: int) -> np.ndarray:
        return self.cnt[p0:p1]

    def sync(self):
        pass
