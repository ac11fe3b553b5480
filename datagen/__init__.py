"""Seeded synthetic inputs (bitvectors, DNA texts with planted repeats, queries,
patterns) shared by the oracle and the GPU path.

Only generation and the documented input encoding live here; no rank or FM
arithmetic.  Everything is deterministic in the seed (counter-based SplitMix64),
so tests and benchmarks can regenerate identical inputs anywhere.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdatagen.so")
_SRC = os.path.join(_HERE, "datagen.c")
_lib = None

u64 = C.c_uint64
u32 = C.c_uint32
dbl = C.c_double
vp = C.c_void_p


def build(force: bool = True) -> str:
    """Compile libdatagen.so with gcc (OpenMP for the large generators)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = C.CDLL(_SO)
        lib.dg_draw.restype = u64
        lib.dg_draw.argtypes = [u64, u64]
        lib.dg_stream.restype = u64
        lib.dg_stream.argtypes = [u64, u64]
        lib.dg_range.restype = u64
        lib.dg_range.argtypes = [u64, u64]
        lib.dg_bits.argtypes = [u64, u32, u64, vp]
        lib.dg_dna_codes.argtypes = [u64, u64, vp]
        lib.dg_plant_repeats.restype = C.c_int
        lib.dg_plant_repeats.argtypes = [u64, vp, u64, u64, u64, u64, dbl]
        lib.dg_pack2.argtypes = [vp, u64, u64, vp]
        lib.dg_bits_tail_garbage.argtypes = [vp, u64, u64]
        lib.dg_queries.argtypes = [u64, u64, u64, vp]
        lib.dg_symbols.argtypes = [u64, u64, vp]
        lib.dg_pattern_offsets.restype = u64
        lib.dg_pattern_offsets.argtypes = [u64, u64, u64, u64, vp]
        lib.dg_pattern_fill.argtypes = [u64, vp, u64, u64, vp, dbl, dbl, vp, vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def draw(seed: int, i: int) -> int:
    return int(_load().dg_draw(seed, i))


def stream(seed: int, tag: int) -> int:
    return int(_load().dg_stream(seed, tag))


def bits(seed: int, n: int, p: float = 0.5, tail_garbage: bool = False) -> np.ndarray:
    """Bernoulli(p) bitvector of n bits as u64 words (ceil(n/64) of them, at least 1).

    p is quantised to a 16-bit threshold: P(1) = round(p * 65536) / 65536."""
    nw = max(1, (n + 63) // 64)
    out = np.empty(nw, dtype=np.uint64)
    thr = int(round(p * 65536))
    thr = min(max(thr, 0), 65536)
    _load().dg_bits(seed, thr, nw, _ptr(out))
    if n % 64:
        out[n // 64] &= np.uint64((1 << (n % 64)) - 1)
    if n == 0:
        out[0] = 0
    if tail_garbage:
        _load().dg_bits_tail_garbage(_ptr(out), n, stream(seed, 99) | 1)
    return out


def dna_codes(seed: int, n: int) -> np.ndarray:
    out = np.empty(max(n, 1), dtype=np.uint8)[:n]
    if n:
        _load().dg_dna_codes(seed, n, _ptr(out))
    return out


def plant_repeats(seed: int, codes: np.ndarray, nseg: int = 1000, seglen: int = 10000, copies: int = 20,
                  sub: float = 0.01) -> np.ndarray:
    """In place; see datagen.c for the planting rule.  Returns codes."""
    assert codes.dtype == np.uint8 and codes.flags["C_CONTIGUOUS"]
    rc = _load().dg_plant_repeats(seed, _ptr(codes), codes.size, nseg, seglen, copies, sub)
    if rc != 0:
        raise ValueError("plant_repeats: text shorter than a segment or out of memory")
    return codes


def pack2(codes: np.ndarray, tail_garbage: bool = False, seed: int = 0) -> np.ndarray:
    n = codes.size
    nw = max(1, (n + 31) // 32)
    out = np.zeros(nw, dtype=np.uint64)
    if n:
        _load().dg_pack2(_ptr(np.ascontiguousarray(codes)), n, (stream(seed, 98) | 1) if tail_garbage else 0,
                         _ptr(out))
    return out


def queries(seed: int, n: int, nq: int) -> np.ndarray:
    """nq positions uniform in [0, n] (inclusive)."""
    out = np.empty(max(nq, 1), dtype=np.uint64)[:nq]
    if nq:
        _load().dg_queries(seed, n, nq, _ptr(out))
    return out


def symbols(seed: int, nq: int) -> np.ndarray:
    out = np.empty(max(nq, 1), dtype=np.uint8)[:nq]
    if nq:
        _load().dg_symbols(seed, nq, _ptr(out))
    return out


def patterns(seed: int, codes: np.ndarray, npat: int, minlen: int = 20, maxlen: int = 250,
             frac_sampled: float = 0.9, sub: float = 0.01):
    """Returns (pat u8 codes, off u64[npat+1], kind u8[npat]).  See datagen.c."""
    off = np.empty(npat + 1, dtype=np.uint64)
    total = int(_load().dg_pattern_offsets(seed, npat, minlen, maxlen, _ptr(off)))
    pat = np.empty(max(total, 1), dtype=np.uint8)
    kind = np.empty(max(npat, 1), dtype=np.uint8)
    src = np.ascontiguousarray(codes) if codes.size else np.zeros(1, dtype=np.uint8)
    if npat:
        _load().dg_pattern_fill(seed, _ptr(src), codes.size, npat, _ptr(off), frac_sampled, sub, _ptr(pat),
                                _ptr(kind))
    return pat[:total], off, kind[:npat]


def arrivals(seed: int, rate: float, count: int) -> np.ndarray:
    """Poisson-process arrival times (seconds) of `count` requests at `rate` per second:
    exponential gaps -ln(1-U)/rate with U from the SplitMix64 stream."""
    s = stream(seed, 21)
    u = np.array([(draw(s, i) >> 11) * (1.0 / 9007199254740992.0) for i in range(count)], dtype=np.float64)
    return np.cumsum(-np.log1p(-u) / rate)


def request_sizes(seed: int, count: int, max_size: int = 4096) -> np.ndarray:
    """Request sizes log-uniform in [1, max_size]: floor(exp(U * ln(max_size+1))), clipped."""
    s = stream(seed, 22)
    u = np.array([(draw(s, i) >> 11) * (1.0 / 9007199254740992.0) for i in range(count)], dtype=np.float64)
    k = np.floor(np.exp(u * np.log(max_size + 1.0))).astype(np.int64)
    return np.clip(k, 1, max_size)
