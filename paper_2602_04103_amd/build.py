"""Compile the HIP sources into the in-tree shared library libquadrank.so (gfx950 only)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libquadrank.so")
ARCH = "gfx950"

SOURCES = ["api.hip", "scan.hip", "birank.hip", "quadrank.hip", "quadfm.hip", "gather.hip", "graph.hip", "serve.hip",
           "sa_device.hip", "bwt_host.cpp"]

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from forming packed fp32 instructions (none are needed here)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


SCRATCH_KERNELS: list = []


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    extra = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    # report kernels that spill to scratch (private memory): every kernel here should use registers only
    name = None
    for line in r.stderr.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split("[")[0].strip()
        elif "ScratchSize" in line and name:
            size = int(line.split(":")[-1].split("[")[0].strip() or 0)
            if size:
                SCRATCH_KERNELS.append((src, name, size))
    return obj


def build() -> str:
    """Compile every source and link libquadrank.so (always rebuilds)."""
    os.makedirs(OUT_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-6000:]))
    os.replace(tmp, LIB)
    for src, name, size in SCRATCH_KERNELS:
        print("warning: %s: kernel %s uses %d bytes of scratch per lane" % (src, name, size))
    return LIB


if __name__ == "__main__":
    print(build())
