"""Autotuner for the query kernels: times candidate launch configurations on the live structure
with the caller's own query batch and keeps the fastest.  Results are cached per
(device, structure kind, size class) in a JSON file so a process tunes each shape once."""
from __future__ import annotations

import json
import os
import statistics

import torch

# lanes per query, queries in flight per lane (pair), threads per workgroup, resident waves per CU,
# and the tile size of the position-ordered (sweep) form
RANK_CANDIDATES = (
    [dict(lanes=2, per_lane=p, block=b, grid_waves=0) for p in (1, 2, 4) for b in (128, 256)]
    + [dict(lanes=2, per_lane=p, block=256, grid_waves=g) for p in (2, 4, 8) for g in (8, 16, 32)]
    + [dict(lanes=1, per_lane=p, block=256, grid_waves=0) for p in (1, 2)]
    + [dict(lanes=2, per_lane=p, block=256, grid_waves=0, sweep=t) for t in (1024, 2048, 4096) for p in (1, 2)]
)
FM_CANDIDATES = [dict(block=b, refill=r, waves_per_cu=w) for b in (64, 256) for r in (8, 32, 64) for w in (8, 12, 16, 20, 24)]

_CACHE_PATH = os.environ.get("QR_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), ".tune_cache.json"))


def _key(kind: str, n: int) -> str:
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return "%s|%s|2^%d" % (name, kind, max(0, n).bit_length())


def _load_cache() -> dict:
    try:
        with open(_CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value) -> None:
    c = _load_cache()
    c[key] = value
    try:
        tmp = _CACHE_PATH + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, _CACHE_PATH)
    except OSError:
        pass


def time_launch(fn, reps: int = 5, stream=None) -> float:
    """Median seconds of fn() over reps, by HIP events on the current stream, after one warm-up."""
    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    return statistics.median(ts)


def tune(kind: str, n: int, set_tuning, run, candidates, reps: int = 5, use_cache: bool = True):
    """Apply and return the fastest candidate; `run` performs one launch with the current setting.
    Returns (best, table) where table lists (candidate, seconds)."""
    key = _key(kind, n)
    if use_cache:
        cached = _load_cache().get(key)
        if cached:
            set_tuning(**cached)
            return cached, []
    table = []
    for cand in candidates:
        set_tuning(**cand)
        table.append((cand, time_launch(run, reps)))
    best = min(table, key=lambda x: x[1])[0]
    set_tuning(**best)
    _store(key, best)
    return best, table
