"""ORACLE — test infrastructure only.

Plain CPU statement of what the GPU path computes (rank, rank4, FM-index
count), written from the QuadRank paper (arXiv 2602.04103).  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the product library never does, and the two share no code.

Functions cite the passage they follow:
  rank_bits  — Section 1 rank definition with sigma = 2, rank(q) = rank(q, 1) (Section 3)
  rank_dna   — Section 1 rank definition rank(q, c) over the DNA alphabet
  rank4_dna  — Section 4: the ranks of all four symbols at one position
  prefix_rank_dna — the count of characters at most c before q (the operation proposed in the
               paper's closing section for a bidirectional FM-index)
  count_*    — Appendix D: count-only exact search; naive, suffix-array and
               textbook backward-search statements of the same count
  check_sa   — whether given row values are the suffix array of T$ (the order the suffix-array
               count searches), by direct comparison of neighbouring suffixes
  locate_sa  — the positions of every occurrence in suffix-array order (the locate query the
               paper's closing section proposes for its FM-index)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None

u64 = C.c_uint64
i64 = C.c_int64
vp = C.c_void_p


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP only over independent queries)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = C.CDLL(_SO)
        lib.or_rank_bits.restype = i64
        lib.or_rank_bits.argtypes = [vp, u64, vp, u64, vp]
        lib.or_rank_dna.restype = i64
        lib.or_rank_dna.argtypes = [vp, u64, vp, vp, u64, vp]
        lib.or_rank4_dna.restype = i64
        lib.or_rank4_dna.argtypes = [vp, u64, vp, u64, vp]
        lib.or_prefix_rank_dna.restype = i64
        lib.or_prefix_rank_dna.argtypes = [vp, u64, vp, vp, u64, vp]
        lib.or_check_sa.restype = C.c_int
        lib.or_check_sa.argtypes = [vp, u64, vp]
        lib.or_count_naive.argtypes = [vp, u64, vp, vp, u64, vp]
        lib.or_suffix_array.argtypes = [vp, u64, vp]
        lib.or_bwt.restype = u64
        lib.or_bwt.argtypes = [vp, u64, vp, vp]
        lib.or_count_sa.argtypes = [vp, u64, vp, vp, vp, u64, vp]
        lib.or_interval_sa.argtypes = [vp, u64, vp, vp, vp, u64, vp, vp]
        lib.or_count_backward.restype = C.c_int
        lib.or_count_backward.argtypes = [vp, u64, vp, vp, u64, vp]
        lib.or_kmer_intervals.restype = C.c_int
        lib.or_kmer_intervals.argtypes = [vp, u64, C.c_int, vp, vp]
        lib.or_set_threads.restype = C.c_int
        lib.or_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Threads used by the query loops from now on (n <= 0 keeps the setting); returns the previous
    count.  Results do not depend on it."""
    return int(_load().or_set_threads(int(n)))


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _nonempty(a: np.ndarray, dtype) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=dtype)
    return a if a.size else np.zeros(1, dtype=dtype)


BAD = np.uint64(0xFFFFFFFFFFFFFFFF)


def rank_bits(words: np.ndarray, n: int, q: np.ndarray) -> np.ndarray:
    """rank(q) = number of 1 bits before position q, 0 <= q <= n (out-of-range q -> 2^64-1)."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.empty(max(q.size, 1), dtype=np.uint64)
    rc = _load().or_rank_bits(_p(_nonempty(words, np.uint64)), n, _p(_nonempty(q, np.uint64)), q.size, _p(out))
    if rc < 0:
        raise MemoryError("oracle rank_bits")
    return out[: q.size]


def rank_dna(packed: np.ndarray, n: int, q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """rank(q, c) = occurrences of symbol c before position q."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.uint8)
    assert q.size == c.size
    out = np.empty(max(q.size, 1), dtype=np.uint64)
    rc = _load().or_rank_dna(_p(_nonempty(packed, np.uint64)), n, _p(_nonempty(q, np.uint64)),
                             _p(_nonempty(c, np.uint8)), q.size, _p(out))
    if rc < 0:
        raise MemoryError("oracle rank_dna")
    return out[: q.size]


def rank4_dna(packed: np.ndarray, n: int, q: np.ndarray) -> np.ndarray:
    """rank4(q) = (rank(q,A), rank(q,C), rank(q,G), rank(q,T)); shape (nq, 4)."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.empty((max(q.size, 1), 4), dtype=np.uint64)
    rc = _load().or_rank4_dna(_p(_nonempty(packed, np.uint64)), n, _p(_nonempty(q, np.uint64)), q.size, _p(out))
    if rc < 0:
        raise MemoryError("oracle rank4_dna")
    return out[: q.size]


def prefix_rank_dna(packed: np.ndarray, n: int, q: np.ndarray, c: np.ndarray) -> np.ndarray:
    """prefix_rank(q, c) = number of characters t_i <= c with i < q (out of range -> 2^64-1)."""
    q = np.ascontiguousarray(q, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.uint8)
    assert q.size == c.size
    out = np.empty(max(q.size, 1), dtype=np.uint64)
    rc = _load().or_prefix_rank_dna(_p(_nonempty(packed, np.uint64)), n, _p(_nonempty(q, np.uint64)),
                                    _p(_nonempty(c, np.uint8)), q.size, _p(out))
    if rc < 0:
        raise MemoryError("oracle prefix_rank_dna")
    return out[: q.size]


def count_naive(text: np.ndarray, pat: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Occurrences of each pattern (CSR: pat codes, off[npat+1]) in text, by direct comparison."""
    npat = off.size - 1
    out = np.empty(max(npat, 1), dtype=np.uint64)
    if npat:
        _load().or_count_naive(_p(_nonempty(text, np.uint8)), text.size, _p(_nonempty(pat, np.uint8)),
                               _p(np.ascontiguousarray(off, dtype=np.uint64)), npat, _p(out))
    return out[:npat]


def suffix_array(text: np.ndarray) -> np.ndarray:
    """Suffix array of text + '$' ('$' smallest), n+1 entries, by comparison sort."""
    n = text.size
    sa = np.empty(n + 1, dtype=np.int64)
    _load().or_suffix_array(_p(_nonempty(text, np.uint8)), n, _p(sa))
    return sa


def check_sa(text: np.ndarray, sa: np.ndarray) -> int:
    """0 if sa (n+1 row values, any integer dtype) is the suffix array of text + '$': a permutation
    of 0..n whose neighbouring rows hold strictly increasing suffixes by direct comparison ('$'
    smallest); 1 if a value is out of range or repeated; 2 if a neighbouring pair is out of order."""
    n = text.size
    s = np.ascontiguousarray(sa, dtype=np.int64)
    if s.size != n + 1:
        return 1
    rc = _load().or_check_sa(_p(_nonempty(text, np.uint8)), n, _p(s))
    if rc < 0:
        raise MemoryError("oracle check_sa")
    return int(rc)


def bwt(text: np.ndarray, sa: np.ndarray):
    """(BWT codes with '$' as 4, row of '$')."""
    n = text.size
    out = np.empty(n + 1, dtype=np.uint8)
    d = _load().or_bwt(_p(_nonempty(text, np.uint8)), n, _p(np.ascontiguousarray(sa, dtype=np.int64)), _p(out))
    return out, int(d)


def count_sa(text: np.ndarray, sa: np.ndarray, pat: np.ndarray, off: np.ndarray) -> np.ndarray:
    npat = off.size - 1
    out = np.empty(max(npat, 1), dtype=np.uint64)
    if npat:
        _load().or_count_sa(_p(_nonempty(text, np.uint8)), text.size, _p(np.ascontiguousarray(sa, dtype=np.int64)),
                            _p(_nonempty(pat, np.uint8)), _p(np.ascontiguousarray(off, dtype=np.uint64)), npat,
                            _p(out))
    return out[:npat]


def interval_sa(text: np.ndarray, sa: np.ndarray, pat: np.ndarray, off: np.ndarray):
    """(lo, hi): the suffix-array range of the suffixes of T$ that start with each pattern."""
    npat = off.size - 1
    lo = np.empty(max(npat, 1), dtype=np.uint64)
    hi = np.empty(max(npat, 1), dtype=np.uint64)
    if npat:
        _load().or_interval_sa(_p(_nonempty(text, np.uint8)), text.size, _p(np.ascontiguousarray(sa, dtype=np.int64)),
                               _p(_nonempty(pat, np.uint8)), _p(np.ascontiguousarray(off, dtype=np.uint64)), npat,
                               _p(lo), _p(hi))
    return lo[:npat], hi[:npat]


def locate_sa(text: np.ndarray, sa: np.ndarray, pat: np.ndarray, off: np.ndarray):
    """locate: the text positions of every occurrence of each pattern, in suffix-array order
    (SA[lo..hi) of the pattern's range).  Returns (start, pos): pattern i owns
    pos[start[i]:start[i+1]].  The empty pattern owns all n+1 suffixes."""
    lo, hi = interval_sa(text, sa, pat, off)
    lens = (hi - lo).astype(np.int64)
    start = np.zeros(lo.size + 1, dtype=np.uint64)
    start[1:] = np.cumsum(lens)
    total = int(start[-1])
    rows = np.repeat(lo.astype(np.int64) - start[:-1].astype(np.int64), lens) + np.arange(total, dtype=np.int64)
    return start, np.asarray(sa, dtype=np.int64)[rows].astype(np.uint64)


def count_backward(bwt_codes: np.ndarray, pat: np.ndarray, off: np.ndarray) -> np.ndarray:
    """Textbook backward search over a BWT with '$' as its own symbol (code 4)."""
    n = bwt_codes.size - 1
    npat = off.size - 1
    out = np.empty(max(npat, 1), dtype=np.uint64)
    if npat:
        rc = _load().or_count_backward(_p(np.ascontiguousarray(bwt_codes, dtype=np.uint8)), n,
                                       _p(_nonempty(pat, np.uint8)), _p(np.ascontiguousarray(off, dtype=np.uint64)),
                                       npat, _p(out))
        if rc:
            raise MemoryError("oracle count_backward")
    return out[:npat]


def revcomp(codes: np.ndarray) -> np.ndarray:
    """Reverse complement of DNA codes (A<->T, C<->G: code c -> 3 - c), read backwards."""
    return (3 - np.asarray(codes, dtype=np.uint8)[::-1]).astype(np.uint8)


def count_both_strands(text: np.ndarray, sa: np.ndarray, pat: np.ndarray, off: np.ndarray) -> np.ndarray:
    """count(P) + count(revcomp(P)) for every pattern (the empty pattern counts n+1 once); codes > 3
    make a pattern count 0 on both strands.  Saturates at 2^32-1 like the u32 result it checks."""
    npat = off.size - 1
    fwd = count_sa(text, sa, pat, off)
    rc = [revcomp(pat[int(off[i]):int(off[i + 1])]) for i in range(npat)]
    for i in range(npat):
        if np.any(pat[int(off[i]):int(off[i + 1])] > 3):
            rc[i] = np.full(max(1, int(off[i + 1] - off[i])), 9, np.uint8)
    roff = np.zeros(npat + 1, np.uint64)
    roff[1:] = np.cumsum([x.size for x in rc])
    rflat = np.concatenate(rc).astype(np.uint8) if rc else np.zeros(0, np.uint8)
    rev = count_sa(text, sa, rflat, roff)
    out = fwd + rev
    out[(off[1:] - off[:-1]) == 0] = text.size + 1
    return np.minimum(out, np.uint64(0xFFFFFFFF))


def kmer_intervals(bwt_codes: np.ndarray, k: int = 8):
    """(lo, hi) arrays of length 4^k: the interval after k backward steps for every k-mer."""
    n = bwt_codes.size - 1
    lo = np.empty(1 << (2 * k), dtype=np.uint64)
    hi = np.empty(1 << (2 * k), dtype=np.uint64)
    rc = _load().or_kmer_intervals(_p(np.ascontiguousarray(bwt_codes, dtype=np.uint8)), n, k, _p(lo), _p(hi))
    if rc:
        raise MemoryError("oracle kmer_intervals")
    return lo, hi
