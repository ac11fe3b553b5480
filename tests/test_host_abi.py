"""CPU checks of the C ABI: the library loads, exports every function include/quadrank.h declares,
its exact line division matches integer division, and host-side argument validation rejects bad
calls before touching the GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "quadrank.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return", "sizeof")))


def test_library_exports_every_declared_symbol():
    import paper_2602_04103_amd as qr
    qr.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", qr.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_line_division_is_exact():
    import paper_2602_04103_amd as qr
    rng = np.random.default_rng(1)
    for which, d, limit in ((0, 1008, 1 << 42), (1, 480, 1 << 44), (2, 992, 1 << 48), (3, 448, 1 << 48),
                            (5, 960, 1 << 48), (6, 384, 1 << 48)):
        xs = list(range(0, 5000)) + [int(x) for x in rng.integers(0, limit, 20000, dtype=np.int64)]
        for k in (1, 2, 63, 64, 127, 128, (limit // d) - 1, (1 << 40) // d, (1 << 62) // d):
            xs += [k * d - 1, k * d, k * d + 1]
        xs += [(1 << 63) - 1]
        for x in xs:
            assert qr.qr_line_of(x, which) == x // d, (which, x)


def test_fm_line_division_32_bit():
    """The FM search's 32-bit line index of every layout it runs on (480, 448 and 384 bases per
    line): the library's form on boundaries and samples, and each constant exhaustively over every
    32-bit position (a small C program)."""
    import shutil
    import tempfile
    import paper_2602_04103_amd as qr
    rng = np.random.default_rng(2)
    forms = ((4, 480, 5, 0x11111112), (7, 448, 6, 0x24924925), (8, 384, 7, 0x55555556))
    for which, d, _, _ in forms:
        xs = list(range(0, 4000)) + [int(x) for x in rng.integers(0, 1 << 32, 50_000, dtype=np.int64)]
        for k in (1, 2, 15, 16, 1 << 20, (1 << 32) // d - 1, (1 << 32) // d):
            xs += [k * d - 1, k * d, k * d + 1]
        xs += [(1 << 32) - 1]
        for x in xs:
            if x < (1 << 32):
                assert qr.qr_line_of(x, which) == x // d, (d, x)
        assert qr.qr_line_of(1 << 32, which) == (1 << 64) - 1
    if shutil.which("gcc") is None:
        pytest.skip("no host compiler for the exhaustive check")
    checks = "\n".join(
        "        if ((uint32_t)((((uint64_t)((uint32_t)x >> %d)) * 0x%xull) >> 32) != (uint32_t)(x / %d)) {\n"
        "            printf(\"%d %%llu\\n\", (unsigned long long)x);\n"
        "            return 1;\n"
        "        }" % (s, m, d, d) for _, d, s, m in forms)
    src = """
#include <stdint.h>
#include <stdio.h>
int main(void) {
    for (uint64_t x = 0; x < (1ull << 32); ++x) {
%s
    }
    return 0;
}
""" % checks
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "div.c"), os.path.join(d, "div")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-O2", "-o", exe, c], check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout


def test_host_argument_validation():
    import paper_2602_04103_amd as qr
    L = qr.lib()
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert L.birank_build(None, 5, None, C.byref(h)) == qr.QR_EINVAL
    assert L.birank_build(fake, (1 << 42), None, C.byref(h)) == qr.QR_ERANGE
    assert L.birank_build(fake, 10, None, None) == qr.QR_EINVAL
    assert L.quadrank_build(None, 5, None, C.byref(h)) == qr.QR_EINVAL
    assert L.quadrank_build(fake, (1 << 44), None, C.byref(h)) == qr.QR_ERANGE
    assert L.birank_build_ex(fake, (1 << 48), qr.QR_LAYOUT_32, None, C.byref(h)) == qr.QR_ERANGE
    assert L.quadrank_build_ex(fake, (1 << 48), qr.QR_LAYOUT_32, None, C.byref(h)) == qr.QR_ERANGE
    assert L.birank_build_ex(fake, 10, 7, None, C.byref(h)) == qr.QR_EINVAL
    assert L.quadrank_build_ex(fake, 10, -1, None, C.byref(h)) == qr.QR_EINVAL
    assert L.birank_layout_kind(None) == -1 and L.quadrank_layout_kind(None) == -1
    assert L.birank_rank(None, fake, 1, fake, None) == qr.QR_EINVAL
    assert L.quadrank_rank(None, fake, fake, 1, fake, None) == qr.QR_EINVAL
    assert L.quadrank_rank4(None, fake, 1, fake, None) == qr.QR_EINVAL
    assert "null" in qr.last_error()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.qr_status_string(s)


def test_gather_bench_argument_validation():
    """The gather microbenchmark rejects bad lane counts, unknown flags and misaligned pointers."""
    import paper_2602_04103_amd as qr
    L = qr.lib()
    f16, f8 = C.c_void_p(0x10000), C.c_void_p(0x10008)  # never dereferenced: validation fails first
    ok = qr.QR_GATHER_NONTEMPORAL | qr.QR_GATHER_STREAM_IO
    for lanes in (0, 3, 16):
        assert L.qr_gather_lanes_bench_ex(f16, 4, f16, 1, lanes, 0, f16, None) == qr.QR_EINVAL
    assert L.qr_gather_lanes_bench_ex(f16, 4, f16, 1, 2, ok + 4, f16, None) == qr.QR_EINVAL
    assert L.qr_gather_lanes_bench_ex(f8, 4, f16, 1, 2, 0, f16, None) == qr.QR_EINVAL   # lines not 16-byte aligned
    assert L.qr_gather_lanes_bench_ex(f16, 0, f16, 1, 2, 0, f16, None) == qr.QR_EINVAL  # no lines
    assert L.qr_gather_lanes_bench_ex(f16, 4, None, 1, 2, 0, f16, None) == qr.QR_EINVAL
    assert L.qr_gather_lanes_bench_ex(f16, 4, f16, 0, 2, ok, f16, None) == qr.QR_OK      # nothing to do
    assert L.qr_gather_bench(f16, 4, f16, 1, 96, f16, None) == qr.QR_EINVAL
