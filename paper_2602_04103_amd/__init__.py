"""Python binding of the MI355X rank library (include/quadrank.h).

Argument marshalling only: torch supplies device memory (tensor.data_ptr())
and the HIP stream (torch.cuda.current_stream().cuda_stream); every step runs
in the HIP kernels of libquadrank.so.  There is no CPU fallback: if the
library is missing, importing the functions raises.

The functions carry the C names (birank_build, birank_rank, quadrank_rank4,
quadfm_count, ...).  BiRank / QuadRank / QuadFm wrap a handle and free it when
collected.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libquadrank.so")

QR_OK, QR_EINVAL, QR_ENOMEM, QR_EHIP, QR_ERANGE, QR_EDEVICE = 0, -1, -2, -3, -4, -5
QUADFM_BOTH_STRANDS = 1
QR_SERVE_CHECK_FREE_MEMORY = 1
QR_SERVE_PACKED_PATTERNS = 2
QR_SERVE_GROW_FROM_FREE_HBM = 4
QR_SERVE_COPY_ENGINE = 8
QR_SERVE_BOTH_STRANDS = 16
QR_LAYOUT_16, QR_LAYOUT_32, QR_LAYOUT_16P, QR_LAYOUT_64, QR_LAYOUT_16X2, QR_LAYOUT_24_8 = 0, 1, 2, 3, 4, 5
LAYOUT_NAMES = {QR_LAYOUT_16: "16", QR_LAYOUT_32: "32", QR_LAYOUT_16P: "16p", QR_LAYOUT_64: "64",
                QR_LAYOUT_16X2: "16x2", QR_LAYOUT_24_8: "24_8"}
LAYOUT_BY_NAME = {v: k for k, v in LAYOUT_NAMES.items()}


def _super_dtype(layout: int):
    """Element type of a layout's offset array (exact u64 offsets, or shifted u32 ones)."""
    import numpy as np
    return np.uint64 if layout in (QR_LAYOUT_32, QR_LAYOUT_24_8) else np.uint32


class QRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (status %d): %s" % (msg, status, last_error()))
        self.status = status


class qr_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("per_lane", C.c_int32), ("grid_waves", C.c_int32), ("lanes", C.c_int32),
                ("sweep", C.c_int32)]


class qr_serve_stats(C.Structure):
    _fields_ = [("batches", C.c_uint64), ("max_inflight", C.c_uint64), ("max_reserved_bytes", C.c_uint64),
                ("wall_s", C.c_double)]


_lib = None
u64, vp, ci = C.c_uint64, C.c_void_p, C.c_int


def lib():
    """Load libquadrank.so (built by __graft_entry__.build() / paper_2602_04103_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libquadrank.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        sig = {
            "qr_status_string": (C.c_char_p, [ci]),
            "qr_last_error": (C.c_char_p, []),
            "qr_version": (C.c_char_p, []),
            "qr_line_of": (u64, [u64, ci]),
            "birank_build": (ci, [vp, u64, vp, C.POINTER(vp)]),
            "birank_build_ex": (ci, [vp, u64, ci, vp, C.POINTER(vp)]),
            "birank_layout_kind": (ci, [vp]),
            "birank_rank": (ci, [vp, vp, u64, vp, vp]),
            "birank_check": (ci, [vp, vp]),
            "birank_free": (ci, [vp]),
            "birank_len": (u64, [vp]),
            "birank_bytes": (u64, [vp]),
            "birank_layout": (ci, [vp, C.POINTER(vp), C.POINTER(u64), C.POINTER(vp), C.POINTER(u64)]),
            "birank_set_tuning": (ci, [vp, C.POINTER(qr_tuning)]),
            "birank_export": (ci, [vp, vp, vp]),
            "quadrank_build": (ci, [vp, u64, vp, C.POINTER(vp)]),
            "quadrank_build_ex": (ci, [vp, u64, ci, vp, C.POINTER(vp)]),
            "quadrank_layout_kind": (ci, [vp]),
            "quadrank_rank": (ci, [vp, vp, vp, u64, vp, vp]),
            "quadrank_rank4": (ci, [vp, vp, u64, vp, vp]),
            "quadrank_prefix_rank": (ci, [vp, vp, vp, u64, vp, vp]),
            "quadrank_check": (ci, [vp, vp]),
            "quadrank_free": (ci, [vp]),
            "quadrank_len": (u64, [vp]),
            "quadrank_bytes": (u64, [vp]),
            "quadrank_layout": (ci, [vp, C.POINTER(vp), C.POINTER(u64), C.POINTER(vp), C.POINTER(u64)]),
            "quadrank_set_tuning": (ci, [vp, C.POINTER(qr_tuning)]),
            "quadrank_export": (ci, [vp, vp, vp]),
            "qr_gather_bench": (ci, [vp, u64, vp, u64, C.c_uint32, vp, vp]),
            "qr_gather_lanes_bench": (ci, [vp, u64, vp, u64, C.c_uint32, vp, vp]),
            "qr_gather_lanes_bench_ex": (ci, [vp, u64, vp, u64, C.c_uint32, C.c_uint32, vp, vp]),
            "qr_server_create": (ci, [vp, ci, u64, u64, C.c_uint32, C.POINTER(vp)]),
            "qr_server_run": (ci, [vp, vp, vp, vp, u64, vp, vp, vp, C.c_double, C.POINTER(qr_serve_stats)]),
            "qr_server_arena_bytes": (u64, [vp]),
            "qr_server_last_run_staged": (C.c_int64, [vp]),
            "qr_server_free": (ci, [vp]),
            "qr_graph_begin": (ci, [vp]),
            "qr_graph_end": (ci, [vp, C.POINTER(vp)]),
            "qr_graph_launch": (ci, [vp, vp]),
            "qr_graph_free": (ci, [vp]),
        }
        optional = {
            "quadfm_bwt_host": (ci, [vp, u64, vp, C.POINTER(u64)]),
            "quadfm_index_host": (ci, [vp, u64, C.c_uint32, vp, C.POINTER(u64), vp, vp]),
            "quadfm_index_device": (ci, [vp, u64, C.c_uint32, vp, C.POINTER(u64), vp, vp, vp, vp]),
            "quadfm_intervals": (ci, [vp, vp, u64, vp, u64, vp, vp]),
            "quadfm_build_ex": (ci, [vp, u64, u64, C.c_uint32, vp, C.POINTER(vp)]),
            "quadfm_build_layout": (ci, [vp, u64, u64, C.c_uint32, ci, vp, C.POINTER(vp)]),
            "quadfm_layout_kind": (ci, [vp]),
            "quadfm_locate_attach": (ci, [vp, vp, vp, u64, C.c_uint32, vp]),
            "quadfm_locate_offsets": (ci, [vp, vp, u64, vp, vp]),
            "quadfm_locate": (ci, [vp, vp, vp, u64, u64, vp, vp]),
            "quadfm_build": (ci, [vp, u64, u64, vp, C.POINTER(vp)]),
            "quadfm_count": (ci, [vp, vp, vp, u64, vp, vp]),
            "quadfm_count_batched": (ci, [vp, vp, vp, u64, u64, vp, vp]),
            "quadfm_count_ws": (ci, [vp, vp, vp, u64, vp, vp, vp]),
            "quadfm_count_ex": (ci, [vp, vp, u64, vp, u64, C.c_uint32, vp, vp, vp]),
            "quadfm_count_noalloc": (ci, [vp, vp, u64, vp, u64, C.c_uint32, vp, vp]),
            "quadfm_count_packed": (ci, [vp, vp, u64, vp, u64, C.c_uint32, vp, vp, vp]),
            "quadfm_count_batched_ex": (ci, [vp, vp, u64, vp, u64, u64, C.c_uint32, vp, vp]),
            "quadfm_check": (ci, [vp, vp]),
            "quadfm_free": (ci, [vp]),
            "quadfm_len": (u64, [vp]),
            "quadfm_bytes": (u64, [vp]),
            "quadfm_set_tuning": (ci, [vp, C.POINTER(qr_tuning)]),
            "quadfm_table": (ci, [vp, C.POINTER(vp), C.POINTER(u64)]),
            "quadfm_export_table": (ci, [vp, vp]),
            "quadfm_c_array": (ci, [vp, vp]),
        }
        for name, (res, args) in list(sig.items()) + list(optional.items()):
            if not hasattr(L, name):
                if name in sig:
                    raise ImportError("libquadrank.so lacks %s" % name)
                continue
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return (lib().qr_last_error() or b"").decode(errors="replace")


def version() -> str:
    return lib().qr_version().decode()


def _check(rc: int, what: str):
    if rc != QR_OK:
        raise QRError(rc, what)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev(t: torch.Tensor, name: str, dtypes, numel=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s must have dtype in %s, got %s" % (name, dtypes, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return t.data_ptr() if t.numel() else 0


W64 = (torch.int64, torch.uint64)
W8 = (torch.uint8,)
W32 = (torch.int32, torch.uint32)


def qr_line_of(x: int, which: int) -> int:
    return int(lib().qr_line_of(x, which))


# ------------------------------------------------------------------------------------------ BiRank
def birank_build(bits: torch.Tensor, n_bits: int, stream=None, layout: int = QR_LAYOUT_16) -> int:
    h = vp()
    _check(lib().birank_build_ex(_dev(bits, "bits", W64, (n_bits + 63) // 64), n_bits, layout, _stream(stream),
                                 C.byref(h)), "birank_build")
    return h.value


def birank_rank(h: int, q: torch.Tensor, out: torch.Tensor, stream=None):
    nq = q.numel()
    _check(lib().birank_rank(h, _dev(q, "q", W64), nq, _dev(out, "out", W64, nq), _stream(stream)), "birank_rank")
    return out


def birank_check(h: int, stream=None):
    _check(lib().birank_check(h, _stream(stream)), "birank_check")


def birank_free(h: int):
    lib().birank_free(h)


# ---------------------------------------------------------------------------------------- QuadRank
def quadrank_build(packed2: torch.Tensor, n: int, stream=None, layout: int = QR_LAYOUT_16) -> int:
    h = vp()
    _check(lib().quadrank_build_ex(_dev(packed2, "packed2", W64, (n + 31) // 32), n, layout, _stream(stream),
                                   C.byref(h)), "quadrank_build")
    return h.value


def quadrank_rank(h: int, q: torch.Tensor, c: torch.Tensor, out: torch.Tensor, stream=None):
    nq = q.numel()
    _check(lib().quadrank_rank(h, _dev(q, "q", W64), _dev(c, "c", W8, nq), nq, _dev(out, "out", W64, nq),
                               _stream(stream)), "quadrank_rank")
    return out


def quadrank_prefix_rank(h: int, q: torch.Tensor, c: torch.Tensor, out: torch.Tensor, stream=None):
    nq = q.numel()
    _check(lib().quadrank_prefix_rank(h, _dev(q, "q", W64), _dev(c, "c", W8, nq), nq, _dev(out, "out", W64, nq),
                                      _stream(stream)), "quadrank_prefix_rank")
    return out


def quadrank_rank4(h: int, q: torch.Tensor, out4: torch.Tensor, stream=None):
    nq = q.numel()
    _check(lib().quadrank_rank4(h, _dev(q, "q", W64), nq, _dev(out4, "out4", W64, 4 * nq), _stream(stream)),
           "quadrank_rank4")
    return out4


def quadrank_check(h: int, stream=None):
    _check(lib().quadrank_check(h, _stream(stream)), "quadrank_check")


def quadrank_free(h: int):
    lib().quadrank_free(h)


def qr_gather_bench(lines: torch.Tensor, n_lines: int, idx: torch.Tensor, bytes_per_query: int, out: torch.Tensor,
                    stream=None):
    nq = idx.numel()
    _check(lib().qr_gather_bench(_dev(lines, "lines", W64 + W8 + W32, n_lines * 16 if lines.element_size() == 8 else 1),
                                 n_lines, _dev(idx, "idx", W64), nq, bytes_per_query, _dev(out, "out", W64, nq),
                                 _stream(stream)), "qr_gather_bench")
    return out


QR_GATHER_NONTEMPORAL = 1
QR_GATHER_STREAM_IO = 2


def qr_gather_lanes_bench(lines: torch.Tensor, n_lines: int, idx: torch.Tensor, lanes: int, out: torch.Tensor,
                          stream=None, flags: int = 0):
    nq = idx.numel()
    _check(lib().qr_gather_lanes_bench_ex(_dev(lines, "lines", W64, n_lines * 16), n_lines, _dev(idx, "idx", W64), nq,
                                          lanes, flags, _dev(out, "out", W64, nq), _stream(stream)),
           "qr_gather_lanes_bench")
    return out


# ------------------------------------------------------------------------------------------ QuadFm
def quadfm_bwt_host(text_codes):
    """Host input preparation: (BWT of T$ packed 2 bits/symbol with '$' stored as A, dollar row)."""
    import numpy as np
    t = np.ascontiguousarray(text_codes, dtype=np.uint8)
    n = t.size
    out = np.zeros(max(1, (n + 1 + 31) // 32), dtype=np.uint64)
    d = u64()
    src = t if n else np.zeros(1, np.uint8)
    _check(lib().quadfm_bwt_host(src.ctypes.data, n, out.ctypes.data, C.byref(d)), "quadfm_bwt_host")
    return out, int(d.value)


def quadfm_index_host(text_codes, rate: int):
    """Host input preparation with the suffix-array sample for locate: (packed BWT, dollar row,
    mark bits u64[ceil((n+1)/64)], samples u32[n // rate + 1])."""
    import numpy as np
    t = np.ascontiguousarray(text_codes, dtype=np.uint8)
    n = t.size
    out = np.zeros(max(1, (n + 1 + 31) // 32), dtype=np.uint64)
    marks = np.zeros(max(1, (n + 1 + 63) // 64), dtype=np.uint64)
    samples = np.zeros(n // rate + 1, dtype=np.uint32)
    d = u64()
    src = t if n else np.zeros(1, np.uint8)
    _check(lib().quadfm_index_host(src.ctypes.data, n, rate, out.ctypes.data, C.byref(d), marks.ctypes.data,
                                   samples.ctypes.data), "quadfm_index_host")
    return out, int(d.value), marks, samples


def quadfm_index_device(text: torch.Tensor, rate: int = 0, stream=None, sa: torch.Tensor | None = None):
    """Device input preparation from n text codes on the device: (packed BWT, dollar row, mark bits,
    samples) as device tensors (the last two None when rate == 0).  With `sa` (n+1 int32 elements
    on the device) the suffix array itself is written there as u32 row values."""
    n = text.numel()
    dev = text.device
    bwt = torch.empty(max(1, (n + 1 + 31) // 32), dtype=torch.int64, device=dev)
    marks = samples = None
    mp = sp = None
    if rate:
        marks = torch.empty(max(1, (n + 1 + 63) // 64), dtype=torch.int64, device=dev)
        samples = torch.empty(n // rate + 1, dtype=torch.int32, device=dev)
        mp, sp = _dev(marks, "marks", W64), _dev(samples, "samples", W32)
    sap = _dev(sa, "sa", W32, n + 1) if sa is not None else None
    d = u64()
    _check(lib().quadfm_index_device(_dev(text, "text", W8) if n else None, n, rate, _dev(bwt, "bwt", W64), C.byref(d),
                                     mp, sp, sap, _stream(stream)), "quadfm_index_device")
    return bwt, int(d.value), marks, samples


def quadfm_build(bwt_packed2: torch.Tensor, n_plus_1: int, dollar_pos: int, stream=None, kmer: int = 8,
                 layout: int = QR_LAYOUT_16) -> int:
    h = vp()
    _check(lib().quadfm_build_layout(_dev(bwt_packed2, "bwt_packed2", W64, (n_plus_1 + 31) // 32), n_plus_1,
                                     dollar_pos, kmer, layout, _stream(stream), C.byref(h)), "quadfm_build")
    return h.value


def _pat(pat: torch.Tensor):
    """(pointer, byte length) of a pattern buffer; the library checks every offset against the length."""
    return _dev(pat, "pat", W8), pat.numel()


def quadfm_count(h: int, pat: torch.Tensor, off: torch.Tensor, count: torch.Tensor, stream=None):
    """quadfm_count through its length-checked form (quadfm_count_ex with the handle's queue head)."""
    return quadfm_count_ex(h, pat, off, count, 0, None, stream)


def quadfm_count_ws(h: int, pat: torch.Tensor, off: torch.Tensor, count: torch.Tensor, workspace: torch.Tensor,
                    stream=None):
    """quadfm_count_ws through its length-checked form (quadfm_count_ex with a caller-owned head)."""
    _dev(workspace, "workspace", W64, 1)
    return quadfm_count_ex(h, pat, off, count, 0, workspace, stream)


def quadfm_count_ex(h: int, pat: torch.Tensor, off: torch.Tensor, count: torch.Tensor, flags: int = 0,
                    workspace: torch.Tensor | None = None, stream=None):
    npat = off.numel() - 1
    ws = _dev(workspace, "workspace", W64, 1) if workspace is not None else None
    pp, pn = _pat(pat)
    _check(lib().quadfm_count_ex(h, pp, pn, _dev(off, "off", W64), npat, flags, _dev(count, "count", W32, npat), ws,
                                 _stream(stream)), "quadfm_count_ex")
    return count


def quadfm_count_packed(h: int, pat2: torch.Tensor, nbases: int, off: torch.Tensor, count: torch.Tensor,
                        flags: int = 0, workspace: torch.Tensor | None = None, stream=None):
    """quadfm_count_ex over 2-bit packed patterns: pat2 holds the stream's u64 words (at least
    ceil(nbases / 32)), off counts bases."""
    npat = off.numel() - 1
    ws = _dev(workspace, "workspace", W64, 1) if workspace is not None else None
    pp = _dev(pat2, "pat2", W64, (nbases + 31) // 32) if nbases else None
    _check(lib().quadfm_count_packed(h, pp, nbases, _dev(off, "off", W64), npat, flags,
                                     _dev(count, "count", W32, npat), ws, _stream(stream)), "quadfm_count_packed")
    return count


def quadfm_count_noalloc(h: int, pat: torch.Tensor, off: torch.Tensor, count: torch.Tensor, flags: int = 0,
                         stream=None):
    """quadfm_count_ex with the queue head in the library's fixed device array: no allocation and no
    workspace; calls that overlap on one device race."""
    npat = off.numel() - 1
    pp, pn = _pat(pat)
    _check(lib().quadfm_count_noalloc(h, pp, pn, _dev(off, "off", W64), npat, flags, _dev(count, "count", W32, npat),
                                      _stream(stream)), "quadfm_count_noalloc")
    return count


def quadfm_count_batched_ex(h: int, pat: torch.Tensor, off: torch.Tensor, batch: int, flags: int, count: torch.Tensor,
                            stream=None):
    npat = off.numel() - 1
    pp, pn = _pat(pat)
    _check(lib().quadfm_count_batched_ex(h, pp, pn, _dev(off, "off", W64), npat, batch, flags,
                                         _dev(count, "count", W32, npat), _stream(stream)), "quadfm_count_batched_ex")
    return count


def quadfm_count_batched(h: int, pat: torch.Tensor, off: torch.Tensor, batch: int, count: torch.Tensor, stream=None):
    """quadfm_count_batched through its length-checked form (quadfm_count_batched_ex, no flags)."""
    return quadfm_count_batched_ex(h, pat, off, batch, 0, count, stream)


def quadfm_intervals(h: int, pat: torch.Tensor, off: torch.Tensor, iv: torch.Tensor, stream=None):
    npat = off.numel() - 1
    pp, pn = _pat(pat)
    _check(lib().quadfm_intervals(h, pp, pn, _dev(off, "off", W64), npat, _dev(iv, "iv", W32, 2 * npat),
                                  _stream(stream)), "quadfm_intervals")
    return iv


def quadfm_locate_attach(h: int, marks: torch.Tensor, samples: torch.Tensor, rate: int, stream=None):
    _check(lib().quadfm_locate_attach(h, _dev(marks, "marks", W64), _dev(samples, "samples", W32), samples.numel(),
                                      rate, _stream(stream)), "quadfm_locate_attach")


def quadfm_locate_offsets(h: int, iv: torch.Tensor, start: torch.Tensor, stream=None):
    npat = iv.numel() // 2
    _check(lib().quadfm_locate_offsets(h, _dev(iv, "iv", W32, 2 * npat), npat, _dev(start, "start", W64, npat + 1),
                                       _stream(stream)), "quadfm_locate_offsets")
    return start


def quadfm_locate(h: int, iv: torch.Tensor, start: torch.Tensor, total: int, pos: torch.Tensor, stream=None):
    npat = iv.numel() // 2
    _check(lib().quadfm_locate(h, _dev(iv, "iv", W32, 2 * npat), _dev(start, "start", W64, npat + 1), npat, total,
                               _dev(pos, "pos", W32, total), _stream(stream)), "quadfm_locate")
    return pos


def quadfm_check(h: int, stream=None):
    _check(lib().quadfm_check(h, _stream(stream)), "quadfm_check")


def quadfm_free(h: int):
    lib().quadfm_free(h)


# ------------------------------------------------------------------------------------------ graphs
class Graph:
    """A captured launch sequence.  Use as:  with qr.Graph(stream) as g: <enqueue-only calls on stream>
    then g.launch() replays it (same pointers, sizes and stream order)."""

    def __init__(self, stream=None):
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.g = None

    def __enter__(self):
        _check(lib().qr_graph_begin(_stream(self.stream)), "qr_graph_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        g = vp()
        rc = lib().qr_graph_end(_stream(self.stream), C.byref(g))
        if exc_type is None:
            _check(rc, "qr_graph_end")
            self.g = g.value
        return False

    def launch(self, stream=None):
        _check(lib().qr_graph_launch(self.g, _stream(stream if stream is not None else self.stream)),
               "qr_graph_launch")

    def free(self):
        if self.g:
            lib().qr_graph_free(self.g)
            self.g = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------------------- wrappers
class _Handle:
    _free = None

    def __init__(self, h: int):
        self.h = h

    def free(self):
        if self.h:
            type(self)._free(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def _tune(self, fn, block=0, per_lane=0, grid_waves=0, lanes=0, sweep=0):
        """Query-kernel launch settings (qr_tuning): threads per workgroup, queries in flight per lane
        (pair), resident waves per CU (0: one pass over the queries), lanes per query (2: lane pairs)
        and the sweep tile (0, or 1024/2048/4096 queries sorted by position per workgroup)."""
        t = qr_tuning(block, per_lane, grid_waves, lanes, sweep)
        _check(fn(self.h, C.byref(t)), "set_tuning")


def _layout(fn, h):
    a, b = vp(), vp()
    na, nb = u64(), u64()
    _check(fn(h, C.byref(a), C.byref(na), C.byref(b), C.byref(nb)), "layout")
    return a.value, na.value, b.value, nb.value


class BiRank(_Handle):
    """Binary rank structure built on the current device from n bits (u64 words, LSB first)."""
    _free = staticmethod(birank_free)

    def __init__(self, bits: torch.Tensor, n_bits: int, stream=None, layout: int = QR_LAYOUT_16):
        super().__init__(birank_build(bits, n_bits, stream, layout))
        self.n = n_bits
        self.layout = layout

    def rank(self, q: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(q.numel(), dtype=torch.int64, device=q.device)
        return birank_rank(self.h, q, out, stream)

    def check(self, stream=None):
        birank_check(self.h, stream)

    def set_tuning(self, **kw):
        self._tune(lib().birank_set_tuning, **kw)

    @property
    def nbytes(self) -> int:
        return int(lib().birank_bytes(self.h))

    def raw_layout(self):
        """(lines_ptr, n_lines, super_ptr, n_super) device pointers of the raw layout."""
        return _layout(lib().birank_layout, self.h)

    def export(self):
        """Host copies (numpy) of the raw layout: (lines u64[n_lines, 16], super[n_super] of the
        layout's offset type)."""
        import numpy as np
        _, nl, _, ns = self.raw_layout()
        lines = np.empty((nl, 16), dtype=np.uint64)
        sup = np.empty(max(ns, 1), dtype=_super_dtype(self.layout))[:ns]
        _check(lib().birank_export(self.h, lines.ctypes.data, sup.ctypes.data), "birank_export")
        return lines, sup


class QuadRank(_Handle):
    """DNA rank structure built from n 2-bit packed bases."""
    _free = staticmethod(quadrank_free)

    def __init__(self, packed2: torch.Tensor, n: int, stream=None, layout: int = QR_LAYOUT_16):
        super().__init__(quadrank_build(packed2, n, stream, layout))
        self.n = n
        self.layout = layout

    def rank(self, q: torch.Tensor, c: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(q.numel(), dtype=torch.int64, device=q.device)
        return quadrank_rank(self.h, q, c, out, stream)

    def rank4(self, q: torch.Tensor, out4: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out4 is None:
            out4 = torch.empty((q.numel(), 4), dtype=torch.int64, device=q.device)
        return quadrank_rank4(self.h, q, out4, stream)

    def prefix_rank(self, q: torch.Tensor, c: torch.Tensor, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
        """Count of characters at most c before each q."""
        if out is None:
            out = torch.empty(q.numel(), dtype=torch.int64, device=q.device)
        return quadrank_prefix_rank(self.h, q, c, out, stream)

    def check(self, stream=None):
        quadrank_check(self.h, stream)

    def set_tuning(self, **kw):
        self._tune(lib().quadrank_set_tuning, **kw)

    @property
    def nbytes(self) -> int:
        return int(lib().quadrank_bytes(self.h))

    def raw_layout(self):
        """(lines_ptr, n_lines, super_ptr, n_super) device pointers of the raw layout."""
        return _layout(lib().quadrank_layout, self.h)

    def export(self):
        """Host copies (numpy): (lines u64[n_lines, 16], super u32 or u64 [n_super, 4])."""
        import numpy as np
        _, nl, _, ns = self.raw_layout()
        lines = np.empty((nl, 16), dtype=np.uint64)
        sup = np.empty((max(ns, 1), 4), dtype=_super_dtype(self.layout))[:ns]
        _check(lib().quadrank_export(self.h, lines.ctypes.data, sup.ctypes.data), "quadrank_export")
        return lines, sup


class QuadFm(_Handle):
    """Count-only FM-index built from a packed BWT of T$ ('$' stored as A at row dollar_pos)."""
    _free = staticmethod(quadfm_free)

    def __init__(self, bwt_packed2: torch.Tensor, n_plus_1: int, dollar_pos: int, stream=None, kmer: int = 8,
                 layout: int = QR_LAYOUT_16):
        super().__init__(quadfm_build(bwt_packed2, n_plus_1, dollar_pos, stream, kmer, layout))
        self.kmer = kmer
        self.layout = layout
        self.n = n_plus_1 - 1

    @classmethod
    def from_text(cls, text_codes, stream=None, locate_rate: int = 0, device_sa: bool = True, kmer: int = 8,
                  layout: int = QR_LAYOUT_16):
        """Suffix array and BWT built on the device (device_sa=False: on the host with SA-IS), then
        the index build over the QuadRank layout `layout`; with locate_rate > 0 also the suffix-array
        sample at that rate, attached for locate."""
        import numpy as np
        n1 = int(np.asarray(text_codes).size) + 1
        if device_sa:
            t = torch.from_numpy(np.ascontiguousarray(text_codes, dtype=np.uint8)).cuda()
            bwt, dollar, marks, samples = quadfm_index_device(t, locate_rate, stream)
            del t
            fm = cls(bwt, n1, dollar, stream, kmer, layout)
            if locate_rate:
                fm.attach_locate(marks, samples, locate_rate, stream)
            return fm
        if not locate_rate:
            bwt, dollar = quadfm_bwt_host(text_codes)
            return cls(torch.from_numpy(bwt.view(np.int64)).cuda(), n1, dollar, stream, kmer, layout)
        bwt, dollar, marks, samples = quadfm_index_host(text_codes, locate_rate)
        fm = cls(torch.from_numpy(bwt.view(np.int64)).cuda(), n1, dollar, stream, kmer, layout)
        fm.attach_locate(torch.from_numpy(marks.view(np.int64)).cuda(), torch.from_numpy(samples.view(np.int32)).cuda(),
                         locate_rate, stream)
        return fm

    def attach_locate(self, marks: torch.Tensor, samples: torch.Tensor, rate: int, stream=None):
        quadfm_locate_attach(self.h, marks, samples, rate, stream)

    def intervals(self, pat: torch.Tensor, off: torch.Tensor, out: torch.Tensor | None = None, stream=None):
        """(npat, 2) u32 (as int32) BWT intervals [sp, ep) of every pattern."""
        if out is None:
            out = torch.empty((off.numel() - 1, 2), dtype=torch.int32, device=off.device)
        return quadfm_intervals(self.h, pat, off, out, stream)

    def locate(self, pat: torch.Tensor, off: torch.Tensor, stream=None):
        """(start, pos): pattern i occurs at text positions pos[start[i]:start[i+1]] (u32 as int32,
        suffix-array order).  Synchronises once to size the output."""
        npat = off.numel() - 1
        iv = self.intervals(pat, off, stream=stream)
        start = torch.empty(npat + 1, dtype=torch.int64, device=off.device)
        quadfm_locate_offsets(self.h, iv, start, stream)
        quadfm_check(self.h, stream)  # the offsets are final once the stream has drained
        total = int(start[npat].item())
        pos = torch.empty(max(total, 1), dtype=torch.int32, device=off.device)[:total]
        if total:
            quadfm_locate(self.h, iv, start, total, pos, stream)
        return start, pos

    def count(self, pat: torch.Tensor, off: torch.Tensor, out: torch.Tensor | None = None, stream=None,
              both_strands: bool = False):
        if out is None:
            out = torch.empty(off.numel() - 1, dtype=torch.int32, device=off.device)
        if both_strands:
            return quadfm_count_ex(self.h, pat, off, out, QUADFM_BOTH_STRANDS, None, stream)
        return quadfm_count(self.h, pat, off, out, stream)

    def count_packed(self, pat2: torch.Tensor, nbases: int, off: torch.Tensor, out: torch.Tensor | None = None,
                     stream=None, both_strands: bool = False):
        """count over 2-bit packed patterns (pat2: u64 words of the base stream; off counts bases)."""
        if out is None:
            out = torch.empty(off.numel() - 1, dtype=torch.int32, device=off.device)
        return quadfm_count_packed(self.h, pat2, nbases, off, out, QUADFM_BOTH_STRANDS if both_strands else 0, None,
                                   stream)

    def count_batched(self, pat: torch.Tensor, off: torch.Tensor, batch: int = 0, out: torch.Tensor | None = None,
                      stream=None, both_strands: bool = False):
        if out is None:
            out = torch.empty(off.numel() - 1, dtype=torch.int32, device=off.device)
        if both_strands:
            return quadfm_count_batched_ex(self.h, pat, off, batch, QUADFM_BOTH_STRANDS, out, stream)
        return quadfm_count_batched(self.h, pat, off, batch, out, stream)

    def check(self, stream=None):
        quadfm_check(self.h, stream)

    def set_tuning(self, block=0, refill=0, waves_per_cu=0):
        self._tune(lib().quadfm_set_tuning, block=block, per_lane=refill, grid_waves=waves_per_cu)

    def c_array(self):
        import numpy as np
        c = np.zeros(4, dtype=np.uint64)
        _check(lib().quadfm_c_array(self.h, c.ctypes.data), "quadfm_c_array")
        return c

    def table(self):
        """(sp, ep) u32 arrays of the 4^k entries of the k-mer start table."""
        import numpy as np
        t = np.zeros(2 * 4 ** self.kmer, dtype=np.uint32)
        _check(lib().quadfm_export_table(self.h, t.ctypes.data), "quadfm_export_table")
        return t[0::2].copy(), t[1::2].copy()

    @property
    def nbytes(self) -> int:
        return int(lib().quadfm_bytes(self.h))
