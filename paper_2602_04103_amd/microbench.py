"""Microbenchmarks behind the query-kernel design choices (run on the GPU; print one line per point).

  python -m paper_2602_04103_amd.microbench gather   random 64/128-byte line gathers vs working set
  python -m paper_2602_04103_amd.microbench rankws   rank / rank4 throughput against structure size
  python -m paper_2602_04103_amd.microbench lanes    BiRank rank on 2^36 bits: one lane per query
                                                     (several 16-byte loads per lane) vs lane pairs
  python -m paper_2602_04103_amd.microbench glanes   whole-line random gathers read by 1/2/4/8 lanes
                                                     per line, against working set
  python -m paper_2602_04103_amd.microbench order    rank time against the order of a batch's queries
                                                     (and the sweep form)
  python -m paper_2602_04103_amd.microbench stream   streaming-bandwidth references and the builds
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _time(fn, reps=5):
    from paper_2602_04103_amd.autotune import time_launch
    return time_launch(fn, reps)


def gather(args):
    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    nq = 1 << 24
    idx = torch.from_numpy(datagen.bits(7, nq * 64).view(np.int64)).cuda()  # raw 64-bit draws
    out = torch.empty(nq, dtype=torch.int64, device="cuda")
    for gib in args.gib:
        nl = int(gib * (1 << 30)) // 128
        buf = torch.ones(nl * 16, dtype=torch.int64, device="cuda")
        for b in (64, 128):
            t = _time(lambda: qr.qr_gather_bench(buf, nl, idx, b, out))
            print("gather ws=%.3f GiB bytes=%d: %.2f G lines/s (%.0f GB/s of 128-byte lines)"
                  % (gib, b, nq / t / 1e9, nq * 128 / t / 1e9), flush=True)
        del buf
        torch.cuda.empty_cache()


def glanes(args):
    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    nq = 1 << 24
    idx = torch.from_numpy(datagen.bits(7, nq * 64).view(np.int64)).cuda()  # raw 64-bit draws
    out = torch.empty(nq, dtype=torch.int64, device="cuda")
    for gib in args.gib:
        nl = int(gib * (1 << 30)) // 128
        buf = torch.ones(nl * 16, dtype=torch.int64, device="cuda")
        for ln in args.lanes:
            t = _time(lambda: qr.qr_gather_lanes_bench(buf, nl, idx, ln, out, flags=args.flags))
            print("glanes ws=%.3f GiB lanes=%d flags=%d: %.2f G lines/s (%.0f GB/s of 128-byte lines)"
                  % (gib, ln, args.flags, nq / t / 1e9, nq * 128 / t / 1e9), flush=True)
        del buf
        torch.cuda.empty_cache()


def lanes(args):
    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    n = 1 << args.log_n
    bits = torch.from_numpy(datagen.bits(3636, n, 0.5).view(np.int64)).cuda()
    h = qr.BiRank(bits, n)
    del bits
    torch.cuda.empty_cache()
    nq = 1 << 24
    q = torch.from_numpy(datagen.queries(3736, n, nq).view(np.int64)).cuda()
    out = torch.empty(nq, dtype=torch.int64, device="cuda")
    for lanes_, pl in ((1, 1), (1, 2), (2, 1), (2, 2)):
        h.set_tuning(lanes=lanes_, per_lane=pl, block=256, grid_waves=0)
        t = _time(lambda: h.rank(q, out))
        print("birank n=2^%d lanes_per_query=%d queries_per_lane=%d: %.2f G q/s" % (args.log_n, lanes_, pl,
                                                                                    nq / t / 1e9), flush=True)


def rankws(args):
    """Rank throughput against structure size (cache-resident to HBM-resident), per inline layout;
    the best of 1 and 2 queries per lane pair is printed."""
    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    nq = 1 << 24
    out = torch.empty(4 * nq, dtype=torch.int64, device="cuda")
    layouts = {16: qr.QR_LAYOUT_16, 32: qr.QR_LAYOUT_32}
    for lg in args.qr_log_n:
        n = 1 << lg
        d = torch.from_numpy(datagen.bits(lg, 2 * n, 0.5).view(np.int64)).cuda()
        q = torch.from_numpy(datagen.queries(lg + 1, n, nq).view(np.int64)).cuda()
        c = torch.from_numpy(datagen.symbols(lg + 2, nq)).cuda()
        for L in args.layouts:
            h = qr.QuadRank(d, n, layout=layouts[L])
            t1 = t4 = float("inf")
            for pl in (1, 2):
                h.set_tuning(lanes=2, per_lane=pl, block=256, grid_waves=0)
                t1 = min(t1, _time(lambda: h.rank(q, c, out[:nq])))
                t4 = min(t4, _time(lambda: h.rank4(q, out)))
            print("quadrank L%d n=2^%d (%.2f GiB): rank %.2f G q/s, rank4 %.2f G q/s"
                  % (L, lg, h.nbytes / 2**30, nq / t1 / 1e9, nq / t4 / 1e9), flush=True)
            h.free()
        del d
        torch.cuda.empty_cache()
    for lg in args.br_log_n:
        n = 1 << lg
        d = torch.from_numpy(datagen.bits(lg, n, 0.5).view(np.int64)).cuda()
        q = torch.from_numpy(datagen.queries(lg + 1, n, nq).view(np.int64)).cuda()
        for L in args.layouts:
            h = qr.BiRank(d, n, layout=layouts[L])
            t = float("inf")
            for pl in (1, 2):
                h.set_tuning(lanes=2, per_lane=pl, block=256, grid_waves=0)
                t = min(t, _time(lambda: h.rank(q, out[:nq])))
            print("birank L%d n=2^%d (%.2f GiB): rank %.2f G q/s" % (L, lg, h.nbytes / 2**30, nq / t / 1e9), flush=True)
            h.free()
        del d
        torch.cuda.empty_cache()


def order(args):
    """Rank time against the order of a batch's queries (2^24 uniform queries, 32-bit layouts):
    uniform; reordered with torch.sort so that the plain kernel sees (a) chunks sorted in place,
    (b) every tile's sorted queries interleaved, as if all workgroups swept their tiles in step,
    (c) the whole batch bucketed by position; the sweep form on the original order; and the cost of
    a random 8-byte scatter of 2^24 results back to query order."""
    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    nq = 1 << 24
    ar = torch.arange(nq, device="cuda", dtype=torch.int64)

    def run(name, h, nbits, q, c, rank4):
        out = torch.empty(nq * (4 if rank4 else 1), dtype=torch.int64, device="cuda")

        def go(qq, cc):
            if rank4:
                h.rank4(qq, out)
            elif c is not None:
                h.rank(qq, cc, out)
            else:
                h.rank(qq, out)

        def timed(label, order):
            qq = q[order].contiguous()
            cc = c[order].contiguous() if c is not None else None
            t = _time(lambda: go(qq, cc), 7)
            print("%s %s: %.3f ms, %.2f G q/s" % (name, label, t * 1e3, nq / t / 1e9), flush=True)

        h.set_tuning(lanes=2, per_lane=1, block=256, grid_waves=0)
        t = _time(lambda: go(q, c), 7)
        print("%s uniform order: %.3f ms, %.2f G q/s" % (name, t * 1e3, nq / t / 1e9), flush=True)
        for lc in (10, 13, 16):
            _, perm = torch.sort(((ar >> lc) << 40) | q)
            timed("chunks of 2^%d sorted in place" % lc, perm)
        for lc in (10, 12, 13):
            _, perm = torch.sort(((ar >> lc) << 40) | q)
            _, inter = torch.sort(((ar & ((1 << lc) - 1)) << 20) | (ar >> lc))
            timed("tiles of 2^%d swept in step" % lc, perm[inter])
        for bits in (6, 8, 12):
            _, perm = torch.sort(q >> (nbits - bits), stable=True)
            timed("batch bucketed by the top %d bits" % bits, perm)
        for tile in (1024, 2048, 4096):
            for pl in (1, 2):
                h.set_tuning(lanes=2, per_lane=pl, sweep=tile)
                t = _time(lambda: go(q, c), 7)
                print("%s sweep form, tile %d, %d per pair: %.3f ms, %.2f G q/s"
                      % (name, tile, pl, t * 1e3, nq / t / 1e9), flush=True)
        h.set_tuning(lanes=2, per_lane=1, block=256, grid_waves=0)
        w = 4 if rank4 else 1
        src = out.view(nq, w)
        dst = torch.empty_like(src)
        _, perm = torch.sort(q)
        t = _time(lambda: dst.index_copy_(0, perm, src), 7)
        print("%s scatter of %d-byte results to query order: %.3f ms" % (name, 8 * w, t * 1e3), flush=True)

    n = 1 << 32
    d = torch.from_numpy(datagen.pack2(datagen.dna_codes(3202, n)).view(np.int64)).cuda()
    h = qr.QuadRank(d, n, layout=qr.QR_LAYOUT_32)
    del d
    q = torch.from_numpy(datagen.queries(11, n, nq).view(np.int64)).cuda()
    c = torch.from_numpy(datagen.symbols(12, nq)).cuda()
    run("quadrank rank 2^32", h, 32, q, c, False)
    run("quadrank rank4 2^32", h, 32, q, None, True)
    h.free()
    torch.cuda.empty_cache()
    nb = 1 << 36
    d = torch.from_numpy(datagen.bits(3636, nb, 0.5).view(np.int64)).cuda()
    hb = qr.BiRank(d, nb, layout=qr.QR_LAYOUT_32)
    del d
    torch.cuda.empty_cache()
    qb = torch.from_numpy(datagen.queries(13, nb, nq).view(np.int64)).cuda()
    run("birank 2^36", hb, 36, qb, None, False)


def stream(args):
    """Streaming bandwidth references for the build kernels: a device copy, a read-only reduction
    and a write-only fill of 4 GiB (HIP events, median of 5), then the BiRank (2^36 bits) and
    QuadRank (2^32 bases) builds; run under rocprofv3 --kernel-trace for the build kernels' times."""
    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    nb = 4 << 30
    src = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    t = _time(lambda: dst.copy_(src))
    print("copy 4 GiB: %.3f ms, %.0f GB/s (read + write)" % (t * 1e3, 2 * nb / t / 1e9), flush=True)
    t = _time(lambda: torch.bitwise_not(src, out=dst))
    print("bitwise_not 4 GiB: %.3f ms, %.0f GB/s (read + write)" % (t * 1e3, 2 * nb / t / 1e9), flush=True)
    acc = torch.empty(1, dtype=torch.int64, device="cuda")
    t = _time(lambda: torch.sum(src, dim=0, out=acc))
    print("sum 4 GiB: %.3f ms, %.0f GB/s (read)" % (t * 1e3, nb / t / 1e9), flush=True)
    t = _time(lambda: dst.fill_(7))
    print("fill 4 GiB: %.3f ms, %.0f GB/s (write)" % (t * 1e3, nb / t / 1e9), flush=True)
    del src, dst
    torch.cuda.empty_cache()
    n = 1 << 36
    d = torch.from_numpy(datagen.bits(3636, n, 0.5).view(np.int64)).cuda()
    for L in (qr.QR_LAYOUT_32, qr.QR_LAYOUT_16):
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = qr.BiRank(d, n, layout=L)
            t1 = time.perf_counter()
            print("birank build 2^36 layout %d: %.2f ms wall" % (16 if L == qr.QR_LAYOUT_16 else 32, (t1 - t0) * 1e3),
                  flush=True)
            h.free()
    del d
    torch.cuda.empty_cache()
    n = 1 << 32
    d = torch.from_numpy(datagen.pack2(datagen.dna_codes(3202, n)).view(np.int64)).cuda()
    for L in (qr.QR_LAYOUT_32, qr.QR_LAYOUT_16):
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = qr.QuadRank(d, n, layout=L)
            t1 = time.perf_counter()
            print("quadrank build 2^32 layout %d: %.2f ms wall" % (16 if L == qr.QR_LAYOUT_16 else 32, (t1 - t0) * 1e3),
                  flush=True)
            h.free()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    g = sub.add_parser("gather")
    g.add_argument("--gib", type=float, nargs="+", default=[0.25, 1, 2, 3, 4, 8])
    gl = sub.add_parser("glanes")
    gl.add_argument("--gib", type=float, nargs="+", default=[0.25, 1, 4, 8, 16])
    gl.add_argument("--lanes", type=int, nargs="+", default=[1, 2, 4, 8], choices=[1, 2, 4, 8])
    gl.add_argument("--flags", type=int, default=0, help="1: non-temporal line loads, 2: non-temporal index loads and result stores")
    l = sub.add_parser("lanes")
    l.add_argument("--log-n", type=int, default=36)
    r = sub.add_parser("rankws")
    r.add_argument("--qr-log-n", type=int, nargs="+", default=[24, 26, 28, 30, 31, 32, 33])
    r.add_argument("--br-log-n", type=int, nargs="+", default=[24, 28, 31, 33, 34, 35, 36])
    r.add_argument("--layouts", type=int, nargs="+", default=[16, 32], choices=[16, 32])
    sub.add_parser("order")
    sub.add_parser("stream")
    a = ap.parse_args(argv)
    {"gather": gather, "glanes": glanes, "lanes": lanes, "rankws": rankws, "order": order, "stream": stream}[a.what](a)


if __name__ == "__main__":
    main()
