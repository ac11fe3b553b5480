"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): the product's host input
preparation (SA-IS, BWT, suffix-array sample) and the oracle's C functions, built with g++/gcc for
the host only and run on inputs of many sizes and shapes, including rejected ones."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
           OMP_NUM_THREADS="2")

needs_gcc = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    return r


@needs_gcc
def test_host_input_preparation_sanitized(tmp_path):
    exe = str(tmp_path / "host_driver")
    run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
         os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
         os.path.join(ROOT, "paper_2602_04103_amd", "csrc", "bwt_host.cpp"), "-o", exe])
    r = run([exe], env=ENV, timeout=300)
    assert "0 failures" in r.stdout


@needs_gcc
def test_oracle_sanitized(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-std=gnu11", *SAN, "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe])
    r = run([exe], env=ENV, timeout=300)
    assert "0 disagreements" in r.stdout
