"""Host logic of bench.py: the single-GPU guard and the batch split of the 10^9-query rows."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "single" in r.stderr.lower()
    assert r.stdout.strip() == ""  # no JSON line


def test_batches_cover_the_queries_once():
    b = bench.batches(10 ** 9, 1 << 24)
    assert len(b) == 60
    assert all(cnt == 1 << 24 for _, cnt in b[:59]) and b[59][1] == 10_144_256
    assert b[0][0] == 0 and all(o1 == o0 + c0 for (o0, c0), (o1, _) in zip(b, b[1:]))
    assert sum(c for _, c in b) == 10 ** 9
    assert bench.batches(5, 8) == [(0, 5)] and bench.batches(0, 8) == []
