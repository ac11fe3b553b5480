"""Helpers for the GPU parity tests: device staging and loud failure when the HIP path is absent."""
import sys

import numpy as np
import torch


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    import paper_2602_04103_amd as qr
    qr.lib()  # raises if libquadrank.so is missing: no fallback path exists
    return qr


def to_dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def to_host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def announce(*parts):
    """Print what the next GPU step is about to run (flushed), so a fault names its case."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def edge_queries(n: int, line: int, mid: int, sb: int) -> np.ndarray:
    """Positions around line starts, line middles and superblock starts, plus 0 and n."""
    pts = {0, n}
    for base in range(0, n + 1, line):
        if base > 3 * sb + 4 * line:
            break
        for d in (-1, 0, 1):
            pts.add(base + d)
            pts.add(base + mid + d)
    for k in range(0, n // sb + 1):
        for d in (-1, 0, 1, line - 1, line):
            pts.add(k * sb + d)
    for d in range(0, min(n, 2 * line) + 1):
        pts.add(n - d)
    return np.array(sorted(p for p in pts if 0 <= p <= n), dtype=np.uint64)
