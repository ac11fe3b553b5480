"""quadfm_count_noalloc (the count entry point that allocates nothing: its queue head lives in a
fixed device array of the library) against quadfm_count_ex on the same inputs, through the C ABI:
two calls in a row, the second with fewer patterns, both bit-identical to the allocating entry
point, and the counts equal to the oracle's.  Named to be collected last: it leaves the library's device array
holding the last call's queue head, which every call resets before use."""
import ctypes as C

import numpy as np
import pytest
import torch

import datagen
import oracle
from tests.gpu_util import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _call(fn, fm, dp, npat_bytes, do, npat, flags, out, stream, ws=None):
    args = [C.c_void_p(fm.h), C.c_void_p(dp.data_ptr()), C.c_uint64(npat_bytes), C.c_void_p(do.data_ptr()),
            C.c_uint64(npat), C.c_uint32(flags), C.c_void_p(out.data_ptr())]
    if ws is not None:
        args.append(C.c_void_p(ws))
    args.append(C.c_void_p(stream))
    return fn(*args)


def test_count_noalloc_matches_count_ex():
    qr = require_gpu()
    lib = qr.lib()
    lib.quadfm_count_noalloc.restype = C.c_int
    n = 300_000
    codes = datagen.dna_codes(7070, n)
    datagen.plant_repeats(7071, codes, nseg=3, seglen=10_000, copies=20, sub=0.01)
    pat, off, _ = datagen.patterns(7072, codes, 40_000)
    announce("count-noalloc", n, off.size - 1)
    fm = qr.QuadFm.from_text(codes)
    sa = oracle.suffix_array(codes)
    stream = torch.cuda.current_stream().cuda_stream
    for npat, flags in ((40_000, 0), (12_345, 0), (30_000, qr.QUADFM_BOTH_STRANDS), (777, 0)):
        o = off[:npat + 1]
        p = pat[:int(o[-1])]
        dp, do = to_dev(p), to_dev(o)
        a = torch.full((npat,), -1, dtype=torch.int32, device="cuda")
        b = torch.full((npat,), -1, dtype=torch.int32, device="cuda")
        assert _call(lib.quadfm_count_ex, fm, dp, p.size, do, npat, flags, a, stream, ws=0) == 0
        assert _call(lib.quadfm_count_noalloc, fm, dp, p.size, do, npat, flags, b, stream) == 0
        fm.check()
        got_a, got_b = a.cpu().numpy().view(np.uint32), b.cpu().numpy().view(np.uint32)
        assert np.array_equal(got_b, got_a), (npat, flags)
        if flags:
            want = oracle.count_both_strands(codes, sa, p, o).astype(np.uint32)
        else:
            want = oracle.count_sa(codes, sa, p, o).astype(np.uint32)
        assert np.array_equal(got_b, want), (npat, flags)
        # the binding's wrapper of the same entry point
        c = qr.quadfm_count_noalloc(fm.h, dp, do, torch.empty(npat, dtype=torch.int32, device="cuda"), flags)
        assert np.array_equal(c.cpu().numpy().view(np.uint32), want), (npat, flags)
    fm.free()


def test_count_noalloc_rejects_bad_arguments():
    qr = require_gpu()
    lib = qr.lib()
    codes = datagen.dna_codes(7073, 5000)
    fm = qr.QuadFm.from_text(codes)
    dp = to_dev(codes[:100].copy())
    do = to_dev(np.array([0, 10, 100], np.uint64))
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    announce("count-noalloc-args")
    assert _call(lib.quadfm_count_noalloc, fm, dp, 100, do, 2, 0x80, out, stream) == qr.QR_EINVAL  # unknown flag
    args = [None, C.c_void_p(dp.data_ptr()), C.c_uint64(100), C.c_void_p(do.data_ptr()), C.c_uint64(2), C.c_uint32(0),
            C.c_void_p(out.data_ptr()), C.c_void_p(stream)]
    assert lib.quadfm_count_noalloc(*args) == qr.QR_EINVAL                                        # no handle
    fm.free()
