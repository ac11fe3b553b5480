"""Serving loop for FM-index count requests against a device-resident QuadFm index.

Continuous batching.  Requests arrive over time, each carrying a block of patterns.  Whenever a
slot is free and device memory allows, every request that has arrived (FIFO, up to a batch limit)
is admitted as one batch:
  - the batch's patterns are moved to device memory taken from an arena (the HBM budget; the native
    loop can grow it from free device memory),
  - the persistent count kernel runs on the slot's own stream with the slot's own queue head,
  - the counts come back to pinned host memory (the native loop stages small batches with kernels
    that read and write the pinned host arrays, and copies larger ones).
Up to `slots` batches are in flight at once, so batches that arrive while others run overlap on the
device.  A request completes when the host observes its batch's completion event; its latency is
completion time minus arrival time.

The scheduler is written against a small executor interface (`submit`, `poll`, `counts`), with the
GPU executor below (the tests drive it with a CPU stand-in of their own).  `NativeServer` runs the
same policy in the library's native loop (qr_server_*), which is what the benchmark measures.
"""
from __future__ import annotations

import bisect
import dataclasses
import time
from typing import Callable, Optional

import numpy as np


# --------------------------------------------------------------------------------------------- arena
class Arena:
    """First-fit allocator over [0, size) with aligned blocks; frees may arrive in any order."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]  # sorted, disjoint, coalesced (start, end)

    def alloc(self, nbytes: int, align: int = 256) -> Optional[int]:
        for k, (a, b) in enumerate(self.free):
            s = (a + align - 1) // align * align
            if s + nbytes <= b:
                pieces = []
                if s > a:
                    pieces.append((a, s))
                if s + nbytes < b:
                    pieces.append((s + nbytes, b))
                self.free[k:k + 1] = pieces
                return s
        return None

    def release(self, start: int, nbytes: int):
        blk = (start, start + nbytes)
        k = bisect.bisect_left(self.free, blk)
        self.free.insert(k, blk)
        merged = []
        for a, b in self.free:
            if merged and merged[-1][1] >= a:
                merged[-1] = (merged[-1][0], max(merged[-1][1], b))
            else:
                merged.append((a, b))
        self.free = merged

    @property
    def free_bytes(self) -> int:
        return sum(b - a for a, b in self.free)


# ------------------------------------------------------------------------------------------ requests
@dataclasses.dataclass
class Workload:
    """All requests of a run as one CSR: request r owns patterns [req_off[r], req_off[r+1]) of
    (pat, off); arrival[r] is its arrival time in seconds from the start."""
    pat: np.ndarray       # u8 codes
    off: np.ndarray       # u64, npat + 1
    req_off: np.ndarray   # i64, nreq + 1
    arrival: np.ndarray   # f64, nreq

    @property
    def nreq(self) -> int:
        return self.arrival.size

    def packed(self) -> np.ndarray:
        """The patterns as one stream of 2-bit codes in u64 words (base i at bits [2 (i mod 32), +2)
        of word i / 32); off then counts bases.  Computed once and kept."""
        if getattr(self, "_pat2", None) is None:
            import datagen
            self._pat2 = datagen.pack2(self.pat)
        return self._pat2

    def batch_bytes(self, r0: int, r1: int) -> int:
        """Arena bytes of a batch of requests [r0, r1) with byte patterns: the pattern bytes from the
        first one's start rounded down to 8, the offsets and the counts, each padded to 256."""
        p0, p1 = int(self.req_off[r0]), int(self.req_off[r1])
        c0, c1 = int(self.off[p0]), int(self.off[p1])
        chars = c1 - c0 // 8 * 8 if c1 > c0 else 0
        return _pad(chars) + _pad(8 * (p1 - p0 + 1)) + _pad(4 * (p1 - p0)) + 256


def _pad(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


def make_workload(seed: int, text_codes: np.ndarray, rate_patterns_per_s: float, duration_s: float,
                  max_requests: int = 200_000, max_size: int = 4096) -> Workload:
    """Poisson arrivals whose request sizes are log-uniform in [1, max_size] patterns; the request rate is
    the pattern rate divided by the mean request size."""
    import datagen
    mean_size = float(np.mean(datagen.request_sizes(seed ^ 0x5EED, 20_000, max_size)))
    req_rate = rate_patterns_per_s / mean_size
    nreq = int(min(max_requests, max(8, np.ceil(req_rate * duration_s))))
    arrival = datagen.arrivals(seed, req_rate, nreq)
    sizes = datagen.request_sizes(seed, nreq, max_size)
    npat = int(sizes.sum())
    pat, off, _ = datagen.patterns(seed + 1, text_codes, npat)
    req_off = np.zeros(nreq + 1, dtype=np.int64)
    req_off[1:] = np.cumsum(sizes)
    return Workload(pat=pat, off=off, req_off=req_off, arrival=arrival - arrival[0])


# ------------------------------------------------------------------------------------------ executors
class GpuExecutor:
    """Runs batches on the GPU: per slot a stream and an 8-byte queue head; device memory for the
    batches comes from one arena buffer of `budget_bytes`."""

    def __init__(self, fm, workload: Workload, slots: int, budget_bytes: int):
        import torch

        import paper_2602_04103_amd as qr
        self.torch, self.qr, self.fm, self.w = torch, qr, fm, workload
        dev = torch.device("cuda")
        self.arena_dev = torch.empty(int(budget_bytes), dtype=torch.uint8, device=dev)
        self.heads = torch.zeros(slots, dtype=torch.int64, device=dev)
        self.streams = [torch.cuda.Stream() for _ in range(slots)]  # default priority
        # pinned host copies of the request stream and of the results
        self.h_pat = torch.from_numpy(workload.pat).pin_memory()
        self.h_cnt = torch.empty(int(workload.off.size - 1), dtype=torch.int32).pin_memory()
        self.events = [None] * slots
        self.jobs = [None] * slots

    def submit(self, slot: int, r0: int, r1: int, base: int):
        torch, w = self.torch, self.w
        p0, p1 = int(w.req_off[r0]), int(w.req_off[r1])
        c0, c1 = int(w.off[p0]), int(w.off[p1])
        npat, chars = p1 - p0, c1 - c0
        o_pat = base
        o_off = base + _pad(chars)
        o_cnt = o_off + _pad(8 * (npat + 1))
        d_pat = self.arena_dev[o_pat:o_pat + max(chars, 1)]
        d_off = self.arena_dev[o_off:o_off + 8 * (npat + 1)].view(torch.int64)
        d_cnt = self.arena_dev[o_cnt:o_cnt + 4 * npat].view(torch.int32)
        h_off = torch.from_numpy((w.off[p0:p1 + 1] - w.off[p0]).astype(np.int64))
        s = self.streams[slot]
        with torch.cuda.stream(s):
            if chars:
                d_pat[:chars].copy_(self.h_pat[c0:c1], non_blocking=True)
            d_off.copy_(h_off.pin_memory(), non_blocking=True)
            self.qr.quadfm_count_ws(self.fm.h, d_pat, d_off, d_cnt, self.heads[slot:slot + 1], stream=s)
            self.h_cnt[p0:p1].copy_(d_cnt, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot] = ev
        self.jobs[slot] = (p0, p1)

    def poll(self, slot: int) -> bool:
        return self.events[slot].query()

    def counts(self, p0: int, p1: int) -> np.ndarray:
        return self.h_cnt[p0:p1].numpy()

    def sync(self):
        self.torch.cuda.synchronize()


# ------------------------------------------------------------------------------------------ native loop
class NativeServer:
    """The same policy run by the library's native loop (qr_server_*): slots, arena budget, batch cap,
    the optional free-memory check, the optional growth of the arena from free device memory
    (`grow`) and optional counts over both strands; host buffers are pinned once per workload."""

    def __init__(self, fm, slots: int, budget_bytes: int, max_batch_patterns: int = 1 << 18,
                 check_free_memory: bool = False, packed: bool = False, grow: bool = False,
                 copy_engine: bool = False, both_strands: bool = False):
        import ctypes as C

        import paper_2602_04103_amd as qr
        self.qr, self.fm, self.packed = qr, fm, packed
        h = C.c_void_p()
        flags = ((qr.QR_SERVE_CHECK_FREE_MEMORY if check_free_memory else 0)
                 | (qr.QR_SERVE_PACKED_PATTERNS if packed else 0) | (qr.QR_SERVE_GROW_FROM_FREE_HBM if grow else 0)
                 | (qr.QR_SERVE_COPY_ENGINE if copy_engine else 0) | (qr.QR_SERVE_BOTH_STRANDS if both_strands else 0))
        qr._check(qr.lib().qr_server_create(fm.h, slots, int(budget_bytes), int(max_batch_patterns), flags,
                                            C.byref(h)), "qr_server_create")
        self.h = h.value
        self.counts_host = None

    def run(self, w: Workload, deadline_s: float = 600.0, pin: bool = True) -> "ServeStats":
        """Serve the workload.  The host buffers are pinned (so batches of up to 4 MiB are staged by
        kernels) unless pin is False, which leaves them pageable and the loop copying."""
        import ctypes as C

        import torch
        qr = self.qr

        def host(a):
            t = torch.from_numpy(a)
            return t.pin_memory() if pin else t.clone()
        if self.packed:  # 2-bit words: a quarter of the bytes to move
            h_pat = host(w.packed().view(np.int64))
        else:
            h_pat = host(w.pat if w.pat.size else np.zeros(1, np.uint8))
        h_off = host(np.ascontiguousarray(w.off, dtype=np.uint64).view(np.int64))
        h_cnt = host(np.zeros(max(1, int(w.off.size - 1)), dtype=np.int32))
        req_off = np.ascontiguousarray(w.req_off, dtype=np.uint64)
        arrival = np.ascontiguousarray(w.arrival, dtype=np.float64)
        finish = np.full(w.nreq, np.nan)
        st = qr.qr_serve_stats()
        qr._check(qr.lib().qr_server_run(self.h, h_pat.data_ptr(), h_off.data_ptr(), req_off.ctypes.data, w.nreq,
                                         arrival.ctypes.data, h_cnt.data_ptr(), finish.ctypes.data, float(deadline_s),
                                         C.byref(st)), "qr_server_run")
        self.counts_host = h_cnt.numpy()[: int(w.off.size - 1)]
        return ServeStats(latency_s=finish - arrival, finish_s=finish, batches=int(st.batches),
                          max_inflight=int(st.max_inflight), max_reserved_bytes=int(st.max_reserved_bytes),
                          patterns=int(w.req_off[-1]), wall_s=float(st.wall_s),
                          req_patterns=np.diff(np.asarray(w.req_off, dtype=np.int64)))

    def counts(self, p0: int, p1: int) -> np.ndarray:
        return self.counts_host[p0:p1]

    @property
    def last_run_staged(self) -> int:
        """Batches of the last run staged by kernels from pinned host memory (the others were
        copied); -1 before the first run."""
        return int(self.qr.lib().qr_server_last_run_staged(self.h)) if self.h else -1

    @property
    def arena_bytes(self) -> int:
        """Device bytes of the arena: the budget, plus the chunks growth has added."""
        return int(self.qr.lib().qr_server_arena_bytes(self.h)) if self.h else 0

    def free(self):
        if self.h:
            self.qr.lib().qr_server_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------ scheduler
@dataclasses.dataclass
class ServeStats:
    latency_s: np.ndarray        # per request
    finish_s: np.ndarray         # per request, from start
    batches: int
    max_inflight: int
    max_reserved_bytes: int
    patterns: int
    wall_s: float
    req_patterns: Optional[np.ndarray] = None  # patterns of each request (for the batch sizes)

    def batch_sizes(self) -> Optional[np.ndarray]:
        """Patterns per batch, recovered from the finish times: a batch's requests are consecutive
        (FIFO admission) and all finish when the host sees that batch complete (batches the host
        sees complete at the same instant count as one)."""
        if self.req_patterns is None or not self.finish_s.size:
            return None
        f = self.finish_s
        starts = np.concatenate([[0], np.nonzero(f[1:] != f[:-1])[0] + 1])
        return np.add.reduceat(self.req_patterns, starts)

    def summary(self) -> dict:
        lat = self.latency_s
        span = float(self.finish_s.max() - 0.0) if lat.size else 0.0
        return {
            "requests": int(lat.size),
            "patterns": int(self.patterns),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
            "patterns_per_s": float(self.patterns / span) if span > 0 else None,
            "batches": self.batches,
            "max_inflight_batches": self.max_inflight,
            "max_reserved_bytes": self.max_reserved_bytes,
            **self._batch_summary(),
        }

    def _batch_summary(self) -> dict:
        b = self.batch_sizes()
        if b is None or not b.size:
            return {}
        lat = self.latency_s
        slow = lat >= np.percentile(lat, 99)   # the requests behind the p99
        f = self.finish_s
        starts = np.concatenate([[0], np.nonzero(f[1:] != f[:-1])[0] + 1])
        owner = np.repeat(np.arange(b.size), np.diff(np.concatenate([starts, [f.size]])))
        return {"batch_patterns_p50": float(np.percentile(b, 50)), "batch_patterns_p99": float(np.percentile(b, 99)),
                "batch_patterns_max": int(b.max()),
                "batch_patterns_of_p99_requests_median": float(np.median(b[owner[slow]]))}


class Server:
    def __init__(self, executor, slots: int, budget_bytes: int, max_batch_patterns: int = 1 << 18,
                 free_bytes_fn: Optional[Callable[[], int]] = None):
        self.ex = executor
        self.slots = slots
        self.arena = Arena(budget_bytes)
        self.max_batch_patterns = max_batch_patterns
        self.free_bytes_fn = free_bytes_fn  # optional extra admission limit (device free memory)

    def run(self, w: Workload, clock: Optional[Callable[[], float]] = None, time_scale: float = 1.0,
            deadline_s: float = 600.0) -> ServeStats:
        """Serve every request of `w`.  `clock` returns seconds since start (real time by default)."""
        if clock is None:
            t0 = time.perf_counter()
            clock = lambda: (time.perf_counter() - t0) * time_scale
        nreq = w.nreq
        finish = np.full(nreq, np.nan)
        free_slots = list(range(self.slots))
        inflight = {}  # slot -> (r0, r1, base, nbytes)
        nxt = 0        # next request not yet admitted (FIFO)
        batches = max_inflight = max_reserved = 0
        reserved = 0
        done = 0
        start = clock()
        while done < nreq:
            now = clock()
            if now - start > deadline_s:
                raise TimeoutError("serving run exceeded its deadline with %d of %d requests done" % (done, nreq))
            progressed = False
            # completions (any order)
            for slot in list(inflight):
                if self.ex.poll(slot):
                    r0, r1, base, nb = inflight.pop(slot)
                    t = clock()
                    finish[r0:r1] = t
                    done += r1 - r0
                    self.arena.release(base, nb)
                    reserved -= nb
                    free_slots.append(slot)
                    progressed = True
            # admissions: all arrived requests, FIFO, as large a batch as slot, arena and limit allow
            while free_slots and nxt < nreq and w.arrival[nxt] <= now:
                r1 = nxt + 1
                arrived = bisect.bisect_right(w.arrival, now, lo=nxt)
                while r1 < arrived and int(w.req_off[r1 + 1] - w.req_off[nxt]) <= self.max_batch_patterns:
                    r1 += 1
                nb = w.batch_bytes(nxt, r1)
                while r1 > nxt + 1 and nb > self.arena.size:
                    r1 -= 1
                    nb = w.batch_bytes(nxt, r1)
                if nb > self.arena.size:
                    raise MemoryError("request %d needs %d bytes, more than the whole budget %d" % (nxt, nb,
                                                                                                  self.arena.size))
                if self.free_bytes_fn is not None and nb > self.free_bytes_fn():
                    break
                base = self.arena.alloc(nb)
                if base is None:
                    break  # wait for memory to free up
                slot = free_slots.pop()
                self.ex.submit(slot, nxt, r1, base)
                inflight[slot] = (nxt, r1, base, nb)
                reserved += nb
                batches += 1
                max_inflight = max(max_inflight, len(inflight))
                max_reserved = max(max_reserved, reserved)
                nxt = r1
                progressed = True
            if not progressed:
                time.sleep(2e-5)
        self.ex.sync()
        lat = finish - w.arrival
        return ServeStats(latency_s=lat, finish_s=finish, batches=batches, max_inflight=max_inflight,
                          max_reserved_bytes=max_reserved, patterns=int(w.req_off[-1]), wall_s=clock() - start)

    def counts_of(self, w: Workload, r: int) -> np.ndarray:
        return self.ex.counts(int(w.req_off[r]), int(w.req_off[r + 1]))
