#!/usr/bin/env python3
"""Benchmark of the rank / FM-index hot path on one MI355X.

One step = one batch (2^24 queries) through every rank row of the scale configuration:
  QuadRank rank(q,c) and rank4(q) on a 2^32-base text (uniform ACGT with 1000 planted 10-kb
  segments x 20 copies, 1% substitutions), BiRank rank(q) on 2^36-bit vectors at densities 0.5
  and 0.05; 10^9 uniform queries per row are issued as 59 batches of 2^24 and one of 10,144,256,
  step k using batch k mod 60.  Inputs and queries are resident in HBM before timing starts.
`value` is rank queries per second over the whole step.  Per-row rates come from HIP events
around each launch on the stream the kernels run on.

The FM-index rows run the batched-count configuration (2^28-base text with the same repeat
planting, 10^7 patterns of length 20..250, 90% sampled with 1% substitutions, 10% iid) with the
persistent work-queue kernel and with one plain launch per batch, in their own timed loop, then
locate every occurrence of every pattern (intervals, output offsets, LF walks over a suffix-array
sample at rate 32).  The CPU baseline times the oracle on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import itertools
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
BATCH = 1 << 24
TOTAL_Q = 10 ** 9

# The roofline counts the algorithmic lines: one random 128-byte line per rank query.  The coalesced
# query and result streams each query also moves are reported beside it, not inside it.
LINE_BYTES = 128
STREAM_BYTES_PER_QUERY = {
    "quadrank_rank": 8 + 1 + 8,
    "quadrank_rank4": 8 + 32,
    "quadrank_prefix_rank": 8 + 1 + 8,
    "birank_rank_p0.5": 8 + 8,
    "birank_rank_p0.05": 8 + 8,
}


# The paper's own measurements, quoted as context (CPU only; it reports no GPU number): its hardware,
# the memory bounds it measured there, and the rank rate they imply (§5 and the appendix on EPYC).
PAPER_CPU_CONTEXT = {
    "hardware": "Intel Core i7-10750H, 6 cores / 12 threads pinned at 3.0 GHz, dual-channel DDR4-3200 "
                "(controller at 2933 MHz); the paper names its random-access throughput as the limit",
    "ram_latency_ns": 80,
    "one_thread_ns_per_random_line": 7.5,
    "all_threads_ns_per_random_line": 2.5,
    "birank16_prefetch_ns_per_query": {"one_thread": 8, "all_threads": 2.5},
    "derived_all_threads_rank_queries_per_s": 4.0e8,
    "quadrank16": "one query per cache line with prefetching; rank4 costs about as much as rank(q,c)",
    "also": "AMD EPYC 9684X (96 cores, 12-channel DDR5): the same trends, 130 ns RAM latency",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def batches(total: int, batch: int):
    out, o = [], 0
    while o < total:
        out.append((o, min(batch, total - o)))
        o += batch
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-fm", action="store_true", help="skip the FM-index rows")
    ap.add_argument("--fm-patterns", type=int, default=10 ** 7)
    ap.add_argument("--fm-reps", type=int, default=3)
    ap.add_argument("--fm-kmers", default="8,10,12", help="start-table sizes to try; the fastest is measured")
    ap.add_argument("--host-sa", action="store_true",
                    help="prepare the FM-index input (suffix array, BWT) with host SA-IS instead of on the device")
    ap.add_argument("--fm-locate-rate", type=int, default=32,
                    help="suffix-array sampling rate of the locate measurement (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving sweep")
    ap.add_argument("--serve-log-n", type=int, default=30, help="log2 of the served text length")
    ap.add_argument("--serve-loads", default="1e4,1e5,1e6,3e6,1e7,3e7,1e8,2e8,4e8,6e8,8e8,1e9",
                    help="offered loads, patterns/s (past 10^8 the 200 000-request cap shortens the run)")
    ap.add_argument("--serve-bytes", action="store_true",
                    help="send the served patterns one byte per base (default: 2-bit packed words); the native "
                         "loop's top load is also run the other way for comparison")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival span per load point")
    ap.add_argument("--serve-kmer", type=int, default=12, help="start-table size of the served index")
    ap.add_argument("--serve-batch-cap-log", type=int, default=20,
                    help="log2 of the most patterns one served batch takes")
    ap.add_argument("--serve-layout", default="32",
                    help="QuadRank layout of the served index (32: the fastest count over the 2^30-base index)")
    ap.add_argument("--no-fm-hbm", action="store_true",
                    help="skip the FM count measurement on the served (HBM-resident) index")
    ap.add_argument("--fm-hbm-patterns", type=int, default=4 * 10 ** 6)
    ap.add_argument("--no-fm-hbm-k8", action="store_true",
                    help="skip the 8-mer start table in the HBM-resident FM row (the served index's k only)")
    ap.add_argument("--fm-layouts", default="16p,32,64,24_8",
                    help="QuadRank layouts besides the 16-bit one to build the FM rows' indexes over (empty: none)")
    ap.add_argument("--serve-python", action="store_true",
                    help="run the sweep with the Python scheduling loop instead of the native one")
    ap.add_argument("--no-tune", action="store_true", help="use default launch settings")
    ap.add_argument("--rows", default="quadrank_rank,quadrank_rank4,birank_rank_p0.5,birank_rank_p0.05",
                    help="comma-separated rank rows of the step; quadrank_prefix_rank is an optional extra row")
    ap.add_argument("--layouts", default="16,32,16p,64,16x2,24_8",
                    help="line layouts to build for each rank row (16x2 is BiRank's only, 24_8 QuadRank's); "
                         "the tuner picks one per row")
    ap.add_argument("--no-extra", action="store_true", help="skip the prefix_rank row timed outside the step")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing of the steps")
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--tuning-from", default=None,
                    help="apply the launch settings recorded in an earlier bench JSON line instead of tuning")
    ap.add_argument("--gather-gib", default="0.25,1,8",
                    help="comma-separated sizes in GiB: measure the random-line gather ceiling over a fresh "
                         "allocation of each size (after the steps; reported under gather_sweep)")
    ap.add_argument("--gather-lanes", default="2",
                    help="lanes per line (1, 2, 4, 8) of the gather sweep: each size is measured with each")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 1 GiB read + 1 GiB write elementwise kernel (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the rank structures and the FM-index have no multi-GPU "
              "path here (they would be replicated per GPU, with the queries split between GPUs)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_2602_04103_amd as qr
    from paper_2602_04103_amd import autotune, profiling

    qr.lib()  # fail loudly when the HIP library is missing
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = [r for r in args.rows.split(",") if r]
    layouts = [x for x in args.layouts.split(",") if x]
    layout_id = qr.LAYOUT_BY_NAME
    qr_layouts = [L for L in layouts if L != "16x2"]    # QuadRank has no 16x2 layout
    br_layouts = [L for L in layouts if L != "24_8"]    # BiRank has no 24_8 layout
    t_setup = time.time()

    def to_dev(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint64:
            a = a.view(np.int64)
        return torch.from_numpy(a).to(dev)

    # ------------------------------------------------------------------ structures + queries
    structs, qsets, builds = {}, {}, {}

    def build_rate(key, in_bytes, out_bytes, secs):
        """Streaming rate of a build: its algorithmic bytes (the packed input read by the count pass
        and again by the line writer, the structure written once) over the host time of the build
        call, which also holds its device allocations and final synchronisation (a lower bound on
        the kernels' own rate)."""
        algo = 2 * in_bytes + out_bytes
        builds[key + "_algorithmic_bytes"] = algo
        builds[key + "_GBps"] = round(algo / secs / 1e9, 1)
        builds[key + "_frac_of_hbm_peak"] = round(algo / secs / 1e9 / HBM_PEAK_GBS, 4)
    packed_q = None
    n_qr = 1 << 32
    if any(r.startswith("quadrank") for r in rows):
        t0 = time.time()
        codes = datagen.dna_codes(3202, n_qr)
        datagen.plant_repeats(3203, codes, nseg=1000, seglen=10_000, copies=20, sub=0.01)
        packed_q = datagen.pack2(codes)
        del codes
        d = to_dev(packed_q)
        log("quadrank text generated %.1fs" % (time.time() - t0))
        structs["quadrank"] = {}
        for L in qr_layouts:  # untimed first builds on 2^20 bases: the first launches load the code
            qr.QuadRank(d, 1 << 20, layout=layout_id[L]).free()
        for L in qr_layouts:
            torch.cuda.synchronize()
            t0 = time.time()
            structs["quadrank"][L] = qr.QuadRank(d, n_qr, layout=layout_id[L])
            builds["quadrank%s_build_s" % L] = time.time() - t0
            builds["quadrank%s_bytes" % L] = structs["quadrank"][L].nbytes
            build_rate("quadrank%s" % L, n_qr // 4, structs["quadrank"][L].nbytes, time.time() - t0)
        del d
        if "quadrank_rank" in rows:
            qsets["quadrank_rank"] = (to_dev(datagen.queries(3204, n_qr, TOTAL_Q)),
                                      to_dev(datagen.symbols(3205, TOTAL_Q)))
        if "quadrank_rank4" in rows:
            qsets["quadrank_rank4"] = (to_dev(datagen.queries(3206, n_qr, TOTAL_Q)), None)
        if "quadrank_prefix_rank" in rows:  # optional row (not in the default step)
            qsets["quadrank_prefix_rank"] = (to_dev(datagen.queries(3207, n_qr, TOTAL_Q)),
                                             to_dev(datagen.symbols(3208, TOTAL_Q)))
    n_br = 1 << 36
    for dens, seed in ((0.5, 3636), (0.05, 3637)):
        row = "birank_rank_p%g" % dens
        if row not in rows:
            continue
        t0 = time.time()
        d = to_dev(datagen.bits(seed, n_br, dens))
        t1 = time.time()
        structs[row] = {}
        for L in br_layouts:  # untimed first builds on 2^20 bits
            qr.BiRank(d, 1 << 20, layout=layout_id[L]).free()
        for L in br_layouts:
            torch.cuda.synchronize()
            t2 = time.time()
            structs[row][L] = qr.BiRank(d, n_br, layout=layout_id[L])
            builds["birank%s_build_p%g_s" % (L, dens)] = time.time() - t2
            builds["birank%s_bytes" % L] = structs[row][L].nbytes
            build_rate("birank%s_p%g" % (L, dens), n_br // 8, structs[row][L].nbytes, time.time() - t2)
        del d
        qsets[row] = (to_dev(datagen.queries(seed + 100, n_br, TOTAL_Q)), None)
        log("%s ready (gen %.1fs)" % (row, t1 - t0))
    torch.cuda.empty_cache()

    outs = torch.empty(BATCH * 4, dtype=torch.int64, device=dev)
    bl = batches(TOTAL_Q, BATCH)

    def row_layouts(row):
        return qr_layouts if row.startswith("quadrank") else br_layouts

    choice = {row: row_layouts(row)[0] for row in rows}  # layout each row runs on (set by the tuner)

    def handle(row, L=None):
        return structs["quadrank" if row.startswith("quadrank") else row][choice[row] if L is None else L]

    def launch(row, k, L=None):
        o, cnt = bl[k % len(bl)]
        q, c = qsets[row]
        h = handle(row, L)
        if row == "quadrank_rank":
            h.rank(q[o:o + cnt], c[o:o + cnt], outs[:cnt])
        elif row == "quadrank_rank4":
            h.rank4(q[o:o + cnt], outs[:4 * cnt])
        elif row == "quadrank_prefix_rank":
            h.prefix_rank(q[o:o + cnt], c[o:o + cnt], outs[:cnt])
        else:
            h.rank(q[o:o + cnt], outs[:cnt])

    # ------------------------------------------------------------------ autotune (untimed)
    tuning, by_layout = {}, {row: {} for row in rows}
    fixed = None
    if args.tuning_from:
        with open(args.tuning_from) as f:
            prev = json.loads(f.readline())
        fixed = {r: v.get("tuning") for r, v in prev.get("rows", {}).items()}
        fixed["_fm"] = (prev.get("fm") or {}).get("tuning")
        args.fm_tuning = fixed["_fm"]
        # the FM rows' other launch settings, by index size, start table and layout
        fm_prev, hbm_prev = prev.get("fm") or {}, ((prev.get("serve") or {}).get("fm_count_hbm") or {})
        args.fm_fixed = {}
        for name, r in (fm_prev.get("by_layout") or {}).items():
            args.fm_fixed["2^28|layout|" + name] = r.get("tuning")
        for k, r in (hbm_prev.get("by_kmer") or {}).items():
            args.fm_fixed["2^30|k|" + k] = r.get("tuning")
        for name, r in (hbm_prev.get("by_layout") or {}).items():
            args.fm_fixed["2^30|layout|" + name] = r.get("tuning")
    for row in rows:
        if fixed and isinstance(fixed.get(row), dict):
            t = dict(fixed[row])
            L = str(t.pop("layout", "16"))
            choice[row] = L if L in row_layouts(row) else row_layouts(row)[0]
            handle(row).set_tuning(**t)
            tuning[row] = t
            continue
        if args.no_tune:
            handle(row).set_tuning(lanes=2, per_lane=1, block=256, grid_waves=0)
            tuning[row] = "default"
            continue
        best_t = None
        # every timed launch of a candidate takes the next full batch, as the timed steps do: replaying
        # one batch leaves its queries and translations cached and can rank candidates differently
        full = [k for k, (_, cnt) in enumerate(bl) if cnt == BATCH]
        turn = itertools.count()
        for L in row_layouts(row):
            h = handle(row, L)
            best, table = autotune.tune("%s|L%s" % (row, L), h.n, h.set_tuning,
                                        lambda r=row, L=L: launch(r, full[next(turn) % len(full)], L),
                                        autotune.RANK_CANDIDATES, use_cache=False)
            t_best = min(t for _, t in table)
            by_layout[row][L] = {"tuned_launch_ms": round(t_best * 1e3, 4), "tuning": best,
                                 "queries_per_s": BATCH / t_best, "structure_bytes": h.nbytes,
                                 "roofline_frac_hbm": BATCH / t_best * LINE_BYTES / 1e9 / HBM_PEAK_GBS}
            log("tuned %s layout %s -> %s %.3f ms (%s)" % (row, L, best, t_best * 1e3,
                                                          ", ".join("%.3f" % (t * 1e3) for _, t in table[:6])))
            if best_t is None or t_best < best_t:
                best_t, choice[row], tuning[row] = t_best, L, best

    def apply(row):
        if tuning.get(row) not in (None, "default"):
            handle(row).set_tuning(**tuning[row])

    if args.calibrate_copy:
        src = torch.zeros(1 << 27, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # ------------------------------------------------------------------ timed steps
    # The timing events are created (first recorded) before the timed region: creating HIP events
    # inside it would put event-pool growth, a host-side stall, between a launch's two records.
    ev_pairs = {row: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(args.steps)] for row in rows}
    for row in rows:
        for a, b in ev_pairs[row]:
            a.record(stream)
            b.record(stream)
    torch.cuda.synchronize()
    ev = {row: [] for row in rows}
    gc.collect()
    for k in range(args.warmup):  # the warm-up steps run right before the timed ones
        for row in rows:
            apply(row)
            launch(row, k)
    torch.cuda.synchronize()
    gc.disable()  # no collector pause between a launch's two event records
    t_start = time.perf_counter()
    host_max = {row: 0.0 for row in rows}  # longest host time spent issuing one launch
    for k in range(args.steps):
        for row in rows:
            h0 = time.perf_counter()
            apply(row)
            a, b = ev_pairs[row][k]
            a.record(stream)
            launch(row, k)
            b.record(stream)
            ev[row].append((a, b, bl[k % len(bl)][1]))
            host_max[row] = max(host_max[row], time.perf_counter() - h0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    gc.enable()
    step_queries = sum(bl[k % len(bl)][1] for k in range(args.steps)) * len(rows)
    row_res = {}
    for row in rows:
        secs = [a.elapsed_time(b) / 1e3 for a, b, _ in ev[row]]
        nq = sum(c for _, _, c in ev[row])
        per_launch = statistics.mean(secs)
        qps = nq / sum(secs)
        achieved = LINE_BYTES * nq / sum(secs) / 1e9
        with_streams = (LINE_BYTES + STREAM_BYTES_PER_QUERY[row]) * nq / sum(secs) / 1e9
        row_res[row] = {
            "queries_per_s": qps,
            "avg_launch_ms": per_launch * 1e3,
            "launch_ms_min_p50_max": [round(min(secs) * 1e3, 4), round(statistics.median(secs) * 1e3, 4),
                                      round(max(secs) * 1e3, 4)],
            "slowest_launch_step": int(max(range(len(secs)), key=lambda i: secs[i])),
            "host_issue_ms_max": round(host_max[row] * 1e3, 4),
            "lines_per_query": 1,
            "roofline_frac_hbm": achieved / HBM_PEAK_GBS,
            "algorithmic_GBps": achieved,
            "stream_bytes_per_query": STREAM_BYTES_PER_QUERY[row],
            "frac_incl_streams": with_streams / HBM_PEAK_GBS,
            "tuning": (dict(tuning[row], layout=choice[row]) if isinstance(tuning.get(row), dict)
                       else tuning.get(row)),
            "layout": choice[row],
            "by_layout": by_layout[row],
        }
        log("%-20s L%s %.2f G q/s  %.3f ms/launch  lines %.1f%% of HBM (%.1f%% with the query/result streams)" % (
            row, choice[row], qps / 1e9, per_launch * 1e3, 100 * achieved / HBM_PEAK_GBS,
            100 * with_streams / HBM_PEAK_GBS))
    ms_per_step = wall / args.steps * 1e3
    value = step_queries / wall if rows else None

    # dominant kernel = largest share of the step's time
    dom = max(rows, key=lambda r: row_res[r]["avg_launch_ms"]) if rows else None
    form = profiling.launch_form(tuning.get(dom)) if dom else None
    traffic = None
    prof_path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        if dom is None:
            raise KeyError("no rank rows")
        prof = json.load(open(prof_path))
        ent = prof.get("kernels", {}).get(profiling.traffic_key(dom, choice[dom], form))
        if ent and profiling.source_hash(ent.get("sources", [])) == ent.get("source_hash"):
            traffic = ent["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    roofline = None if dom is None else {
        "bound": "hbm",
        "kernel": "%s<%s> (%s)" % (profiling.ROW_KERNELS[dom][form], profiling.layout_token(dom, choice[dom]), dom),
        "row": dom,
        "layout": choice[dom],
        "achieved": round(row_res[dom]["algorithmic_GBps"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(row_res[dom]["roofline_frac_hbm"], 4),
        "traffic": traffic,
        "bytes_per_query": LINE_BYTES,
        "stream_bytes_per_query": STREAM_BYTES_PER_QUERY[dom],
        "frac_incl_streams": round(row_res[dom]["frac_incl_streams"], 4),
    }
    # context for each row's rate: the random-line gather rate over the row's own structure allocation
    # (same size, same pages), two lanes per line, with the non-temporal index and result streams of
    # the rank kernels; the rate a rank kernel would reach if its one random line per query were its
    # only cost (untimed region, after the steps).  Where in HBM an allocation lands moves this rate
    # by several per cent, so each row is compared with its own.
    draws = torch.randint(-2 ** 63, 2 ** 63 - 1, (BATCH,), dtype=torch.int64, device=dev)
    for row in rows:
        lines_ptr, n_lines, _, _ = handle(row).raw_layout()

        def gather():
            rc = qr.lib().qr_gather_lanes_bench_ex(lines_ptr, n_lines, draws.data_ptr(), BATCH, 2,
                                                   qr.QR_GATHER_STREAM_IO, outs.data_ptr(), stream.cuda_stream)
            if rc:
                raise RuntimeError("qr_gather_lanes_bench_ex failed: %d" % rc)

        ceiling = BATCH / autotune.time_launch(gather, reps=7)
        row_res[row]["line_gather_ceiling_lines_per_s"] = round(ceiling, 1)
        row_res[row]["frac_of_line_gather_ceiling"] = round(row_res[row]["queries_per_s"] / ceiling, 4)
        log("%s: %.2f G q/s against %.2f G random lines/s over the same allocation (%.1f%%)" % (
            row, row_res[row]["queries_per_s"] / 1e9, ceiling / 1e9, 100 * row_res[row]["queries_per_s"] / ceiling))
    del draws
    if roofline is not None:
        roofline["line_gather_ceiling"] = {
            "lines_per_s": row_res[dom]["line_gather_ceiling_lines_per_s"],
            "queries_per_s": round(row_res[dom]["queries_per_s"], 1),
            "frac": row_res[dom]["frac_of_line_gather_ceiling"],
            "what": "2^24 uniform random 128-byte lines of the same structure allocation, two lanes per "
                    "line, non-temporal index and result streams (qr_gather_lanes_bench_ex)",
        }

    # ------------------------------------------------------------------ gather ceilings by working set
    gather_sweep = None
    if args.gather_gib:
        gather_sweep = []
        for gib in (float(x) for x in args.gather_gib.split(",") if x):
            for lanes in (int(x) for x in args.gather_lanes.split(",") if x):
                lps = gather_ceiling(qr, torch, dev, int(gib * (1 << 30)), lanes=lanes)
                gather_sweep.append({"gib": gib, "lanes": lanes, "lines_per_s": lps, "GBps_of_lines": lps * 128 / 1e9})
                log("gather ceiling over %.2f GiB, %d lanes per line: %.2f G lines/s (%.0f GB/s of lines)" % (
                    gib, lanes, lps / 1e9, lps * 128 / 1e9))

    # ------------------------------------------------------------------ the same steps from a HIP graph
    # the K timed steps (every row, every batch) captured once and replayed with one launch
    graph_res = None
    if not args.no_graph and rows:
        gs = torch.cuda.Stream()
        g = qr.Graph(gs)
        with torch.cuda.stream(gs):
            with g:
                for k in range(args.steps):
                    for row in rows:
                        apply(row)  # the launch settings are frozen into the captured launches
                        launch(row, k)
        g.launch(gs)  # untimed first replay
        gs.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.launch(gs)
        gs.synchronize()
        t_g = time.perf_counter() - t0
        g.free()
        graph_res = {"rank_queries_per_s": step_queries / t_g, "ms_per_step": t_g / args.steps * 1e3,
                     "launches": args.steps * len(rows)}
        log("graph replay of the %d steps: %.2f G q/s (%.3f ms/step)" % (args.steps, step_queries / t_g / 1e9,
                                                                      t_g / args.steps * 1e3))

    # ------------------------------------------------------------------ extra rows (not in the step)
    # prefix_rank(q, c) on the QuadRank row's queries, structure and launch settings
    extra = {}
    if not args.no_extra and "quadrank_rank" in qsets:
        h = handle("quadrank_rank")
        apply("quadrank_rank")
        q, c = qsets["quadrank_rank"]
        evs = []
        for k in range(args.warmup + args.steps):
            o, cnt = bl[k % len(bl)]
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            h.prefix_rank(q[o:o + cnt], c[o:o + cnt], outs[:cnt])
            b.record(stream)
            if k >= args.warmup:
                evs.append((a, b, cnt))
        torch.cuda.synchronize()
        secs = sum(a.elapsed_time(b) / 1e3 for a, b, _ in evs)
        nq = sum(c_ for _, _, c_ in evs)
        achieved = LINE_BYTES * nq / secs / 1e9
        extra["quadrank_prefix_rank"] = {"queries_per_s": nq / secs, "avg_launch_ms": secs / len(evs) * 1e3,
                                         "roofline_frac_hbm": achieved / HBM_PEAK_GBS, "algorithmic_GBps": achieved,
                                         "layout": choice["quadrank_rank"], "in_step": False}
        log("%-20s L%s %.2f G q/s  %.3f ms/launch  %.1f%% of HBM roofline (outside the step)" % (
            "quadrank_prefix_rank", choice["quadrank_rank"], nq / secs / 1e9, secs / len(evs) * 1e3,
            100 * achieved / HBM_PEAK_GBS))

    # ------------------------------------------------------------------ FM-index rows
    fm_res = None
    if not args.no_fm:
        fm_res = bench_fm(args, qr, autotune, datagen, np, torch, dev, to_dev)
    fm_cpu_inputs = fm_res.pop("_cpu_inputs", None) if fm_res else None

    # ------------------------------------------------------------------ serving sweep
    serve_res = None
    if not args.no_serve:
        serve_res = bench_serve(args, qr, datagen, np, torch, to_dev)

    # ------------------------------------------------------------------ CPU baseline (oracle)
    cpu = None
    if not args.no_cpu_baseline and packed_q is not None and "quadrank_rank" in qsets:
        cpu = cpu_baseline(packed_q, n_qr, datagen, np, with_birank="birank_rank_p0.5" in rows, fm_inputs=fm_cpu_inputs)
        log("cpu baseline (oracle, %d threads, %s): rank %.1f M q/s (one thread %.1f), rank4 %.1f M q/s%s%s" % (
            cpu["cores"], cpu["cpu_model"], cpu["value"] / 1e6, cpu["one_thread_queries_per_s"] / 1e6,
            cpu["rank4_queries_per_s"] / 1e6,
            ", BiRank %.1f M q/s" % (cpu["birank_queries_per_s"] / 1e6) if "birank_queries_per_s" in cpu else "",
            ", FM count %.2f M patterns/s" % (cpu["fm_count_patterns_per_s"] / 1e6)
            if "fm_count_patterns_per_s" in cpu else ""))
    del fm_cpu_inputs

    out = {
        "metric": "rank queries/s + % HBM random-line roofline; FM count patterns/s, p99 latency",
        "value": value,
        "unit": "rank queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "scale rank rows: QuadRank rank(q,c)+rank4 on 2^32 bases (uniform ACGT, 1000 planted "
                        "10-kb segments x20, 1% subs) and BiRank rank on 2^36 bits (Bernoulli 0.5 and 0.05); "
                        "10^9 uniform queries per row in batches of 2^24",
            "global_batch": BATCH,
            "rows_per_step": rows,
            "queries_per_step": step_queries // args.steps,
        },
        "rows": row_res,
        "extra_rows": extra,
        "graph": graph_res,
        "builds": builds,
        "roofline": roofline,
        "gather_sweep": gather_sweep,
        "fm": fm_res,
        "serve": serve_res,
        "cpu_baseline": cpu,
        "paper_cpu_context": PAPER_CPU_CONTEXT,
        "setup_s": round(time.time() - t_setup, 1),
    }
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def bench_fm(args, qr, autotune, datagen, np, torch, dev, to_dev):
    n = 1 << 28
    t0 = time.time()
    codes = datagen.dna_codes(2828, n)
    datagen.plant_repeats(2829, codes, nseg=1000, seglen=10_000, copies=20, sub=0.01)
    t1 = time.time()
    rate = args.fm_locate_rate
    if args.host_sa:
        if rate:
            bwt, dollar, marks, samples = qr.quadfm_index_host(codes, rate)
            marks, samples = to_dev(marks), torch.from_numpy(samples.view(np.int32)).to(dev)
        else:
            bwt, dollar = qr.quadfm_bwt_host(codes)
        bwt = to_dev(bwt)
    else:
        d_text = torch.from_numpy(codes).to(dev)
        # the suffix array is handed out only for the CPU baseline's oracle search (outside the timings)
        d_sa = None if args.no_cpu_baseline else torch.empty(n + 1, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t1 = time.time()
        bwt, dollar, marks, samples = qr.quadfm_index_device(d_text, rate, sa=d_sa)
        del d_text
    t2 = time.time()
    kmers = [int(x) for x in args.fm_kmers.split(",") if x]
    fms = {k: qr.QuadFm(bwt, n + 1, dollar, kmer=k) for k in kmers}
    torch.cuda.synchronize()
    t3 = time.time()
    pat, off, kind = datagen.patterns(2830, codes, args.fm_patterns)
    cpu_inputs = None
    if not args.no_cpu_baseline and not args.host_sa:
        sample = min(args.fm_patterns, 3 * 10 ** 6)  # the oracle's sample: the first 3*10^6 patterns
        cpu_inputs = (codes, d_sa.cpu().numpy().view(np.uint32).astype(np.int64), pat[:int(off[sample])],
                      off[:sample + 1].copy())
        del d_sa
    del codes
    dp, do = to_dev(pat), to_dev(off)
    npat = args.fm_patterns
    # start-table size: the count rate of each k (default launch settings); the fastest is used below
    cnt = torch.empty(npat, dtype=torch.int32, device=dev)
    by_kmer = {k: npat / autotune.time_launch(lambda f=f: f.count(dp, do, cnt), reps=2) for k, f in fms.items()}
    kbest = max(by_kmer, key=by_kmer.get)
    log("fm start table: " + ", ".join("k=%d %.1f M patterns/s" % (k, v / 1e6) for k, v in by_kmer.items()))
    fm = fms.pop(kbest)
    for f in fms.values():
        f.free()
    names = [name for name in args.fm_layouts.split(",") if name]
    others = {name: qr.QuadFm(bwt, n + 1, dollar, kmer=kbest, layout=qr.LAYOUT_BY_NAME[name])
              for name in (["16"] + names if names else [])}
    count_bytes = fm.nbytes
    if rate:
        fm.attach_locate(marks, samples, rate)
        del marks, samples
    del bwt
    total_chars = int(off[-1])
    log("fm index: text %.1fs, %s SA+BWT %.2fs, device build %.2fs" % (t1 - t0, "host" if args.host_sa else "device",
                                                                       t2 - t1, t3 - t2))
    cnt_b = torch.empty(npat, dtype=torch.int32, device=dev)
    if isinstance(getattr(args, "fm_tuning", None), dict):
        best = args.fm_tuning
        fm.set_tuning(**best)
    elif not args.no_tune:
        sub = min(npat, 2_000_000)
        best, _ = autotune.tune("quadfm", n, fm.set_tuning, lambda: fm.count(dp, do[:sub + 1], cnt[:sub]),
                                autotune.FM_CANDIDATES, reps=2, use_cache=False)
    else:
        best = "default"
    t_p = autotune.time_launch(lambda: fm.count(dp, do, cnt), reps=args.fm_reps)
    res = {"workload": "QuadFm count: 2^28-base text (uniform ACGT, 1000 planted 10-kb segments x20, 1%% subs) "
                       "+ sentinel; %d patterns, lengths 20..250, 90%% sampled with 1%% substitutions, 10%% iid"
                       % npat,
           "persistent_patterns_per_s": npat / t_p, "persistent_ms": t_p * 1e3, "tuning": best,
           "index_bytes": count_bytes, "bits_per_base": count_bytes * 8 / n, "pattern_chars": total_chars,
           "sa_bwt_s": t2 - t1, "sa_bwt_on": "host" if args.host_sa else "device",
           "device_build_s_all_kmers": t3 - t2, "kmer": kbest, "by_kmer_patterns_per_s": by_kmer}
    for batch in (1 << 16, 1 << 20, 0):
        t_b = autotune.time_launch(lambda: fm.count_batched(dp, do, batch, cnt_b), reps=args.fm_reps)
        res["batched_%s_patterns_per_s" % (batch or "all")] = npat / t_b
        res["batched_%s_ms" % (batch or "all")] = t_b * 1e3
    best_b = max(v for k, v in res.items() if k.startswith("batched_") and k.endswith("per_s"))
    res["gain_vs_best_batched"] = res["persistent_patterns_per_s"] / best_b
    res["gain_vs_batch_2^16"] = res["persistent_patterns_per_s"] / res["batched_65536_patterns_per_s"]
    res["persistent_equals_batched"] = bool(torch.equal(cnt, cnt_b))
    # both strands: every pattern and its reverse complement, one persistent launch
    cnt2 = torch.empty(npat, dtype=torch.int32, device=dev)
    t_2 = autotune.time_launch(lambda: fm.count(dp, do, cnt2, both_strands=True), reps=args.fm_reps)
    res["both_strands_patterns_per_s"] = npat / t_2
    res["both_strands_ms"] = t_2 * 1e3
    log("fm both strands %.1f M patterns/s (%.2f ms)" % (npat / t_2 / 1e6, t_2 * 1e3))
    # the same count over 2-bit packed patterns (a quarter of the pattern bytes)
    dp2 = to_dev(datagen.pack2(pat))
    cnt3 = torch.empty(npat, dtype=torch.int32, device=dev)
    t_k = autotune.time_launch(lambda: fm.count_packed(dp2, int(off[-1]), do, cnt3), reps=args.fm_reps)
    res["packed_patterns_per_s"] = npat / t_k
    res["packed_equals_bytes"] = bool(torch.equal(cnt3, cnt))
    del dp2, cnt3
    log("fm packed patterns %.1f M patterns/s (%.2f ms), equal=%s" % (npat / t_k / 1e6, t_k * 1e3,
                                                                     res["packed_equals_bytes"]))
    # roofline of the persistent kernel: algorithmic lines (128 B each) per pattern from a sample
    work = fm_work_sample(fm, pat, off, npat, np, torch, to_dev, kmer=kbest)
    achieved = npat / t_p * work["lines_per_pattern"] * 128 / 1e9
    res["work"] = work
    line_bytes = ((n + 1) // 480 + 1) * 128
    ceil_lps = gather_ceiling(qr, torch, dev, line_bytes)
    lps = npat / t_p * work["lines_per_pattern"]
    plps = res["packed_patterns_per_s"] * work["lines_per_pattern"]
    res["roofline"] = {"bound": "cache", "kernel": "fm_persistent_kernel<QR16, false, false, false>",
                       "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac_of_hbm_peak": round(achieved / HBM_PEAK_GBS, 4),
                       "lines_per_s": lps, "line_gather_ceiling_lines_per_s": ceil_lps,
                       "frac": round(lps / ceil_lps, 4),
                       "packed_patterns_lines_per_s": plps, "packed_patterns_frac": round(plps / ceil_lps, 4),
                       "note": "algorithmic 128-byte lines; the %.0f MB of lines fit the 256 MB memory-side cache, "
                               "so the fraction is taken against the measured random-line gather rate over an "
                               "allocation of the same size, not against HBM (which a cache-resident count with "
                               "packed patterns can exceed)" % (line_bytes / 1e6)}
    log("fm work: %.1f steps, %.1f lines, %.1f half lines per pattern -> %.0f GB/s of lines (%.0f%% of HBM), "
        "%.2f G lines/s against a gather ceiling of %.2f G lines/s over %.0f MB (%.0f%%)" % (
            work["steps_per_pattern"], work["lines_per_pattern"], work["half_lines_per_pattern"], achieved,
            100 * achieved / HBM_PEAK_GBS, lps / 1e9, ceil_lps / 1e9, line_bytes / 1e6, 100 * lps / ceil_lps))
    log("fm persistent %.1f M patterns/s; batched best %.1f M; gain %.2fx; equal=%s" % (
        npat / t_p / 1e6, best_b / 1e6, res["gain_vs_best_batched"], res["persistent_equals_batched"]))
    if others:
        ref = cnt.clone()
        res["by_layout"] = fm_layout_rows(args, qr, autotune, np, torch, dev, to_dev, others, ref, dp, do, cnt, pat,
                                          off, npat, n, kbest, min(npat, 2_000_000))
        res["best_layout"], _ = fm_best_layout(res["by_layout"])
        for f in others.values():
            f.free()
    if rate:
        # locate every occurrence of every pattern: intervals, output offsets, then the LF walks
        iv = torch.empty((npat, 2), dtype=torch.int32, device=dev)
        start = torch.empty(npat + 1, dtype=torch.int64, device=dev)
        t_iv = autotune.time_launch(lambda: fm.intervals(dp, do, iv), reps=args.fm_reps)
        t_off = autotune.time_launch(lambda: qr.quadfm_locate_offsets(fm.h, iv, start), reps=args.fm_reps)
        total = int(start[npat].item())
        pos = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
        t_loc = autotune.time_launch(lambda: qr.quadfm_locate(fm.h, iv, start, total, pos), reps=args.fm_reps)
        fm.check()
        res.update({"locate_rate": rate, "locate_sample_bytes": fm.nbytes - count_bytes, "locate_positions": total,
                    "intervals_ms": t_iv * 1e3, "locate_offsets_ms": t_off * 1e3, "locate_ms": t_loc * 1e3,
                    "locate_positions_per_s": total / t_loc,
                    "locate_patterns_per_s_end_to_end": npat / (t_iv + t_off + t_loc),
                    "intervals_sizes_equal_counts": bool(torch.equal(iv[:, 1] - iv[:, 0], cnt))})
        log("fm locate (rate %d): %d positions, %.1f M positions/s; intervals %.2f ms, offsets %.2f ms, walks %.2f ms"
            % (rate, total, total / t_loc / 1e6, t_iv * 1e3, t_off * 1e3, t_loc * 1e3))
    fm.free()
    res["_cpu_inputs"] = cpu_inputs  # taken out by main() for the CPU baseline, not reported
    return res


def gather_ceiling(qr, torch, dev, nbytes, draws=1 << 24, reps=5, lanes=2):
    """Random 128-byte lines per second over a fresh allocation of `nbytes` (2^24 uniform lines, read
    by `lanes` lanes per line, non-temporal index and result streams): the rate a kernel that reads
    one random line per unit of work over a structure of that size can reach."""
    from paper_2602_04103_amd import autotune
    n_lines = max(1, nbytes // 128)
    buf = torch.ones(n_lines * 16, dtype=torch.int64, device=dev)
    idx = torch.randint(-2 ** 63, 2 ** 63 - 1, (draws,), dtype=torch.int64, device=dev)
    out = torch.empty(draws, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def run():
        rc = qr.lib().qr_gather_lanes_bench_ex(buf.data_ptr(), n_lines, idx.data_ptr(), draws, lanes,
                                               qr.QR_GATHER_STREAM_IO, out.data_ptr(), stream.cuda_stream)
        if rc:
            raise RuntimeError("qr_gather_lanes_bench_ex failed: %d" % rc)

    t = autotune.time_launch(run, reps=reps)
    del buf, idx, out
    return draws / t


def bench_fm_hbm(args, qr, autotune, datagen, np, torch, dev, to_dev, text, bwt, dollar, fm_serve):
    """The persistent count on the index the serving sweep uses (2^30 bases: its lines and start
    table exceed the 256 MB memory-side cache, so most line reads go to HBM), against one launch per
    batch, at the start-table size of the batched row (k = 8) and of the served index, over the
    served index's layout; then the same count over every layout (by_layout), whose fastest gives
    the row's roofline."""
    n = text.size
    npat = args.fm_hbm_patterns
    pat, off, _ = datagen.patterns(4040, text, npat)
    dp, do = to_dev(pat), to_dev(off)
    cnt = torch.empty(npat, dtype=torch.int32, device=dev)
    cnt_b = torch.empty(npat, dtype=torch.int32, device=dev)
    line_bytes = ((n + 1) // FM_GEOMETRY[args.serve_layout][0] + 1) * 128
    ceil_lps = gather_ceiling(qr, torch, dev, line_bytes)
    res = {"layout": args.serve_layout,
           "workload": "QuadFm count on the 2^%d-base serving text (uniform ACGT, 1000 planted 10-kb segments x20, "
                       "1%% subs) + sentinel; %d patterns, lengths 20..250, 90%% sampled with 1%% substitutions, "
                       "10%% iid" % (int(np.log2(n)), npat),
           "line_bytes": line_bytes, "line_gather_ceiling_lines_per_s": ceil_lps, "by_kmer": {}}
    fms = {args.serve_kmer: fm_serve}
    if args.serve_kmer != 8 and not args.no_fm_hbm_k8:
        fms[8] = qr.QuadFm(bwt, n + 1, dollar, kmer=8, layout=qr.LAYOUT_BY_NAME[args.serve_layout])
    for k, fm in sorted(fms.items()):
        # the persistent kernel's launch settings tuned on this index (an HBM-resident index wants
        # more patterns in flight than the cache-resident one), on the first 10^6 patterns
        sub = min(npat, 1_000_000)
        best = fm_tune(args, autotune, "2^%d|k|%d" % (int(np.log2(n)), k), n, fm,
                       lambda f=fm: f.count(dp, do[:sub + 1], cnt[:sub]))
        t_p = autotune.time_launch(lambda f=fm: f.count(dp, do, cnt), reps=args.fm_reps)
        row = {"index_bytes": fm.nbytes, "persistent_patterns_per_s": npat / t_p, "persistent_ms": t_p * 1e3,
               "tuning": best}
        dp2, cnt3 = to_dev(datagen.pack2(pat)), torch.empty(npat, dtype=torch.int32, device=dev)
        t_k = autotune.time_launch(lambda f=fm: f.count_packed(dp2, int(off[-1]), do, cnt3), reps=args.fm_reps)
        row["packed_patterns_per_s"] = npat / t_k
        row["packed_equals_bytes"] = bool(torch.equal(cnt3, cnt))
        del dp2, cnt3
        for batch in (1 << 16, 1 << 20, 0):
            t_b = autotune.time_launch(lambda f=fm: f.count_batched(dp, do, batch, cnt_b), reps=args.fm_reps)
            row["batched_%s_patterns_per_s" % (batch or "all")] = npat / t_b
        best_b = max(v for kk, v in row.items() if kk.startswith("batched_"))
        row["gain_vs_best_batched"] = row["persistent_patterns_per_s"] / best_b
        row["persistent_equals_batched"] = bool(torch.equal(cnt, cnt_b))
        work = fm_work_sample(fm, pat, off, npat, np, torch, to_dev, kmer=k, layout=args.serve_layout)
        lps = npat / t_p * work["lines_per_pattern"]
        row["work"] = work
        row["roofline"] = {"bound": "hbm",
                           "kernel": "fm_persistent_kernel<%s, false, false, false>" % FM_TRAIT[args.serve_layout],
                           "achieved": round(lps * 128 / 1e9, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(lps * 128 / 1e9 / HBM_PEAK_GBS, 4),
                           "lines_per_s": lps, "frac_of_line_gather_ceiling": round(lps / ceil_lps, 4)}
        res["by_kmer"][str(k)] = row
        log("fm 2^%d k=%d: persistent %.1f M patterns/s (packed patterns %.1f M), best batched %.1f M (gain %.2fx), "
            "%.1f lines/pattern, %.0f GB/s of lines = %.1f%% of HBM, %.0f%% of the gather ceiling (%.2f G lines/s), "
            "equal=%s" % (
                int(np.log2(n)), k, npat / t_p / 1e6, row["packed_patterns_per_s"] / 1e6, best_b / 1e6,
                row["gain_vs_best_batched"], work["lines_per_pattern"], lps * 128 / 1e9,
                100 * lps * 128 / 1e9 / HBM_PEAK_GBS, 100 * lps / ceil_lps, ceil_lps / 1e9,
                row["persistent_equals_batched"] and row["packed_equals_bytes"]))
        if k != args.serve_kmer:
            fm.free()
        else:
            fm.set_tuning(block=64, refill=32, waves_per_cu=8)  # the serving loop's own settings
    names = [name for name in args.fm_layouts.split(",") if name]
    if names:
        k = args.serve_kmer
        res["by_layout_kmer"] = k
        ref = cnt.clone()
        others = {name: qr.QuadFm(bwt, n + 1, dollar, kmer=k, layout=qr.LAYOUT_BY_NAME[name])
                  for name in ["16"] + names}
        res["by_layout"] = fm_layout_rows(args, qr, autotune, np, torch, dev, to_dev, others, ref, dp, do, cnt, pat,
                                          off, npat, n, k, min(npat, 1_000_000))
        res["best_layout"], res["roofline"] = fm_best_layout(res["by_layout"])
        for f in others.values():
            f.free()
    res["reads_150"] = fm_reads_row(args, autotune, datagen, np, torch, dev, to_dev, text, fm_serve,
                                    res["by_kmer"].get(str(args.serve_kmer), {}).get("tuning"))
    fm_serve.set_tuning(block=64, refill=32, waves_per_cu=8)  # back to the serving loop's settings
    return res


def fm_reads_row(args, autotune, datagen, np, torch, dev, to_dev, text, fm, tuning):
    """The paper's read-counting shape on the served index: 10^6 reads of 150 bases with 1 %
    substitutions, every other one taken from the reverse strand, counted on both strands (and on
    the forward strand alone), with byte and with 2-bit packed reads."""
    nr, rl = 10 ** 6, 150
    rpat, roff, _ = datagen.patterns(4141, text, nr, minlen=rl, maxlen=rl, frac_sampled=1.0, sub=0.01)
    rows = rpat.reshape(nr, rl)
    rows[1::2] = 3 - rows[1::2, ::-1]  # reverse complements
    drp, dro, dr2 = to_dev(rpat), to_dev(roff), to_dev(datagen.pack2(rpat))
    if tuning:
        fm.set_tuning(**tuning)
    c_b = torch.empty(nr, dtype=torch.int32, device=dev)
    c_p = torch.empty(nr, dtype=torch.int32, device=dev)
    t_b = autotune.time_launch(lambda: fm.count(drp, dro, c_b, both_strands=True), reps=args.fm_reps)
    t_p = autotune.time_launch(lambda: fm.count_packed(dr2, nr * rl, dro, c_p, both_strands=True), reps=args.fm_reps)
    both = c_p.cpu().numpy()
    equal = bool(torch.equal(c_b, c_p))
    t_f = autotune.time_launch(lambda: fm.count_packed(dr2, nr * rl, dro, c_p), reps=args.fm_reps)
    fwd = c_p.cpu().numpy()
    row = {"workload": "10^6 reads of 150 bases sampled from the served text with 1% substitutions, every other "
                       "one reverse-complemented",
           "both_strands_reads_per_s": nr / t_b, "both_strands_packed_reads_per_s": nr / t_p,
           "forward_packed_reads_per_s": nr / t_f, "packed_equals_bytes": equal,
           "reads_matched_both_strands": float((both > 0).mean()), "reads_matched_forward": float((fwd > 0).mean())}
    log("fm reads (150 bases, 1%% subs, half reverse strand): both strands %.1f M reads/s (packed %.1f M), forward "
        "only %.1f M; %.1f%% of the reads occur exactly (%.1f%% on the forward strand), equal=%s" % (
            nr / t_b / 1e6, nr / t_p / 1e6, nr / t_f / 1e6, 100 * row["reads_matched_both_strands"],
            100 * row["reads_matched_forward"], equal))
    return row


def fm_tune(args, autotune, key, n, fm, run):
    """The FM count's launch settings: those of --tuning-from's run for this key if it has them, else
    tuned now on the caller's run."""
    t = (getattr(args, "fm_fixed", None) or {}).get(key)
    if isinstance(t, dict):
        fm.set_tuning(**t)
        return t
    best, _ = autotune.tune("quadfm|" + key, n, fm.set_tuning, run, autotune.FM_CANDIDATES, reps=2, use_cache=False)
    return best


# bases per line and header slots of each QuadRank layout the FM-index runs on, and its trait's name
FM_GEOMETRY = {"16": (480, 32), "16p": (480, 32), "32": (448, 64), "64": (384, 128), "24_8": (384, 128)}
FM_TRAIT = {"16": "QR16", "16p": "QR16P", "32": "QR32", "64": "QR64", "24_8": "QR24_8"}


def fm_layout_rows(args, qr, autotune, np, torch, dev, to_dev, fms, ref, dp, do, cnt, pat, off, npat, n, kmer,
                   tune_sub):
    """The persistent count of the same BWT's index over each QuadRank layout (size against
    throughput, as the paper compares QuadFm over each rank structure): tuned launch settings, rate
    with byte patterns and with 2-bit packed ones, counts equal to the reference counts, lines per
    pattern in the layout's geometry and the fraction of the random-line gather ceiling over an
    allocation of the layout's line bytes.  All indexes are built before any is timed, and the rates
    are timed twice, in opposite orders (the best of the two is reported): where an allocation lands
    in HBM moves a random-line rate by a few per cent."""
    import datagen
    rows, rates, prates = {}, {name: [] for name in fms}, {name: [] for name in fms}
    dp2 = to_dev(datagen.pack2(pat))
    nb = int(off[-1])
    for name, fm in fms.items():
        best = fm_tune(args, autotune, "2^%d|layout|%s" % (int(np.log2(n)), name), n, fm,
                       lambda f=fm: f.count(dp, do[:tune_sub + 1], cnt[:tune_sub]))
        rows[name] = {"tuning": best}
    for order in (list(fms), list(fms)[::-1]):
        for name in order:
            rates[name].append(npat / autotune.time_launch(lambda f=fms[name]: f.count(dp, do, cnt), reps=args.fm_reps))
            eq = bool(torch.equal(cnt, ref))
            prates[name].append(npat / autotune.time_launch(lambda f=fms[name]: f.count_packed(dp2, nb, do, cnt),
                                                            reps=args.fm_reps))
            eq = eq and bool(torch.equal(cnt, ref))
            rows[name]["equal_to_reference"] = rows[name].get("equal_to_reference", True) and eq
    del dp2
    for name, fm in fms.items():
        rate, prate = max(rates[name]), max(prates[name])
        work = fm_work_sample(fm, pat, off, npat, np, torch, to_dev, kmer=kmer, layout=name)
        data = FM_GEOMETRY[name][0]
        line_bytes = ((n + 1) // data + 1) * 128
        ceil_lps = gather_ceiling(qr, torch, dev, line_bytes)
        lps, plps = rate * work["lines_per_pattern"], prate * work["lines_per_pattern"]
        rows[name].update({"index_bytes": fm.nbytes, "bits_per_base": round(fm.nbytes * 8 / n, 3),
                           "persistent_patterns_per_s": rate, "passes_patterns_per_s": rates[name],
                           "persistent_ms": npat / rate * 1e3, "packed_patterns_per_s": prate,
                           "packed_passes_patterns_per_s": prates[name],
                           "lines_per_pattern": work["lines_per_pattern"],
                           "half_lines_per_pattern": work["half_lines_per_pattern"], "lines_per_s": lps,
                           "packed_lines_per_s": plps, "line_gather_ceiling_lines_per_s": ceil_lps,
                           "frac_of_line_gather_ceiling": round(lps / ceil_lps, 4),
                           "packed_frac_of_line_gather_ceiling": round(plps / ceil_lps, 4)})
        log("fm 2^%d k=%d layout %s: %.1f M patterns/s, packed %.1f M (passes %s / %s), %.3f bits/base, "
            "%.1f lines/pattern, %.0f%% / %.0f%% of the gather ceiling (%.2f G lines/s), equal=%s" % (
                int(np.log2(n)), kmer, name, rate / 1e6, prate / 1e6,
                " ".join("%.1f" % (r / 1e6) for r in rates[name]), " ".join("%.1f" % (r / 1e6) for r in prates[name]),
                fm.nbytes * 8 / n, work["lines_per_pattern"], 100 * lps / ceil_lps, 100 * plps / ceil_lps,
                ceil_lps / 1e9, rows[name]["equal_to_reference"]))
    return rows


def fm_best_layout(rows):
    """The layout with the highest count rate over packed patterns, and a roofline object for its
    kernel (the served index's form)."""
    name = max(rows, key=lambda k: rows[k]["packed_patterns_per_s"])
    r = rows[name]
    achieved = r["packed_lines_per_s"] * 128 / 1e9
    return name, {"bound": "hbm", "kernel": "fm_persistent_kernel<%s, false, false, true>" % FM_TRAIT[name],
                  "layout": name, "patterns": "2-bit packed", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "lines_per_s": r["packed_lines_per_s"],
                  "frac_of_line_gather_ceiling": r["packed_frac_of_line_gather_ceiling"]}


def fm_work_sample(fm, pat, off, npat, np, torch, to_dev, kmer=8, sample=2000, seed=11, layout="16"):
    """Backward steps, lines and half-line loads per pattern, on a sample of the workload: the
    search of P starts from the interval of its last K = kmer characters and step k (k = 1..m-K)
    turns the interval of the suffix P[m-K-k+1..m) into that of P[m-K-k..m), stopping once it is
    empty.  A step reads one 128-byte line when sp and ep share a line (else two), and one 64-byte
    half when they share a half line (else two halves), in the line geometry of the index's QuadRank
    layout.  The suffix intervals come from quadfm_intervals."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(npat, min(sample, npat), replace=False))
    sufs, owner = [], []
    for p in idx:
        P = pat[int(off[p]):int(off[p + 1])]
        m = P.size
        for k in range(0, m - kmer + 1):  # suffix lengths K..m
            sufs.append(P[m - kmer - k:])
            owner.append(p)
    soff = np.zeros(len(sufs) + 1, np.uint64)
    soff[1:] = np.cumsum([x.size for x in sufs])
    iv = fm.intervals(to_dev(np.concatenate(sufs)), to_dev(soff)).cpu().numpy().view(np.uint32).astype(np.int64)
    DATA, HDR = FM_GEOMETRY[layout]
    MID = 256
    steps = lines = halves = 0
    i = 0
    for p in idx:
        m = int(off[p + 1] - off[p])
        k_max = m - kmer
        for k in range(1, k_max + 1):
            sp, ep = iv[i + k - 1]
            if ep <= sp:
                break
            js, je = sp // DATA, ep // DATA
            hs, he = (sp - js * DATA + HDR) >= MID, (ep - je * DATA + HDR) >= MID
            steps += 1
            lines += 1 if js == je else 2
            halves += 1 if (js == je and hs == he) else 2
        i += k_max + 1
    n = idx.size
    return {"sample_patterns": int(n), "steps_per_pattern": steps / n, "lines_per_pattern": lines / n,
            "half_lines_per_pattern": halves / n}


def serve_light_load(qr, np, torch, to_dev, fm, text, slots, budget, packed):
    """Where a lightly loaded server's latency goes.  Device time of one count of a single pattern
    against its length: the patterns are substrings of the text, so each search takes every step, one
    dependent half-line load per base beyond the start table, and the slope is the latency of one
    step.  Then the native loop on requests of one such pattern arriving once per millisecond (no
    queueing): its latency less the device time is the loop's own cost (copies, launches, polling)."""
    from paper_2602_04103_amd.serve import NativeServer, Workload
    rng = np.random.default_rng(6060)
    n = text.size
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    lens = (20, 80, 160, 250)
    dev_us = {}
    for L in lens:
        pat = np.concatenate([text[p:p + L] for p in rng.integers(0, n - L, 16)])
        dp = to_dev(pat)
        ts = []
        for i in range(16):
            do = to_dev(np.array([i * L, (i + 1) * L], np.uint64))
            fm.count(dp, do, cnt)
            for _ in range(3):
                s.record()
                fm.count(dp, do, cnt)
                e.record()
                e.synchronize()
                ts.append(s.elapsed_time(e) * 1e3)
        dev_us[L] = statistics.median(ts)
    k = fm.kmer
    res = {"single_pattern_device_us": {str(L): round(dev_us[L], 1) for L in lens},
           "us_per_step": round((dev_us[lens[-1]] - dev_us[lens[0]]) / (lens[-1] - lens[0]), 3),
           "start_table_k": k, "one_pattern_requests": {}}
    for L in (20, 250):
        nreq = 200
        pat = np.concatenate([text[p:p + L] for p in rng.integers(0, n - L, nreq)])
        w = Workload(pat=pat, off=np.arange(nreq + 1, dtype=np.uint64) * L, req_off=np.arange(nreq + 1, dtype=np.int64),
                     arrival=np.arange(nreq, dtype=np.float64) * 1e-3)
        srv = NativeServer(fm, slots=slots, budget_bytes=budget, packed=packed)
        srv.run(w, deadline_s=60.0)
        lat = srv.run(w, deadline_s=60.0).latency_s * 1e6
        direct = fm.count(to_dev(w.pat), to_dev(w.off)).cpu().numpy().view(np.uint32)
        res["one_pattern_requests"][str(L)] = {
            "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
            "loop_us_over_device": round(float(np.percentile(lat, 50)) - dev_us[L], 1),
            "equal_to_direct_count": bool(np.array_equal(srv.counts(0, nreq), direct))}
        srv.free()
    log("serve light load: one pattern %s us (%.2f us per step); one-pattern requests p50 %s" % (
        res["single_pattern_device_us"], res["us_per_step"],
        {L: v["p50_us"] for L, v in res["one_pattern_requests"].items()}))
    return res


def bench_serve(args, qr, datagen, np, torch, to_dev):
    """Poisson request arrivals against a device-resident index; each request holds 1..4096 patterns
    (log-uniform), lengths 20..250; offered loads swept; latency from arrival to counts on the host."""
    from paper_2602_04103_amd.serve import GpuExecutor, NativeServer, Server, make_workload
    n = 1 << args.serve_log_n
    t0 = time.time()
    text = datagen.dna_codes(3030, n)
    datagen.plant_repeats(3031, text, nseg=1000, seglen=10_000, copies=20, sub=0.01)
    if args.host_sa:
        bwt, dollar = qr.quadfm_bwt_host(text)
        bwt = to_dev(bwt)
    else:
        bwt, dollar, _, _ = qr.quadfm_index_device(torch.from_numpy(text).cuda(), 0)
    t1 = time.time()
    fm = qr.QuadFm(bwt, n + 1, dollar, kmer=args.serve_kmer, layout=qr.LAYOUT_BY_NAME[args.serve_layout])
    hbm_row = None
    if not args.no_fm_hbm:
        from paper_2602_04103_amd import autotune
        hbm_row = bench_fm_hbm(args, qr, autotune, datagen, np, torch, torch.device("cuda"), to_dev, text, bwt,
                               dollar, fm)
    del bwt
    torch.cuda.empty_cache()
    fm.set_tuning(block=64, refill=32, waves_per_cu=8)
    log("serve index 2^%d: text + %s SA+BWT %.1fs" % (args.serve_log_n, "host" if args.host_sa else "device", t1 - t0))
    slots, budget, cap = 4, 256 << 20, 1 << args.serve_batch_cap_log
    free, total = torch.cuda.mem_get_info()
    res = {"workload": "QuadFm serving: 2^%d-base text (uniform ACGT, 1000 planted 10-kb segments x20, 1%% subs); "
                       "Poisson arrivals, request size log-uniform 1..4096 patterns, lengths 20..250"
                       % args.serve_log_n,
           "slots": slots, "hbm_budget_bytes": budget, "arena": "grows from free HBM (native loop)",
           "batch_cap_patterns": cap,
           "kmer": args.serve_kmer, "layout": args.serve_layout,
           "pattern_form": "bytes" if args.serve_bytes else "packed",
           "device_free_bytes_at_start": int(free),
           "text_sa_bwt_s": t1 - t0, "sa_bwt_on": "host" if args.host_sa else "device", "loads": [],
           "fm_count_hbm": hbm_row}
    # warm-up (untimed): first launches, pinned-memory pools, stream creation
    w0 = make_workload(4999, text, 1e6, 0.05, max_requests=200)
    ex0 = GpuExecutor(fm, w0, slots=slots, budget_bytes=budget)
    Server(ex0, slots=slots, budget_bytes=budget).run(w0, deadline_s=60.0)
    del ex0
    ns0 = NativeServer(fm, slots=slots, budget_bytes=budget)
    ns0.run(w0, deadline_s=60.0)
    ns0.free()
    res["loop"] = "python" if args.serve_python else "native"
    res["light_load"] = serve_light_load(qr, np, torch, to_dev, fm, text, slots, budget, not args.serve_bytes)
    for k, load in enumerate(float(x) for x in args.serve_loads.split(",") if x):
        w = make_workload(5000 + k, text, load, args.serve_seconds, max_requests=200_000)
        if args.serve_python:
            ex = GpuExecutor(fm, w, slots=slots, budget_bytes=budget)
            srv = Server(ex, slots=slots, budget_bytes=budget, max_batch_patterns=cap,
                         free_bytes_fn=lambda: torch.cuda.mem_get_info()[0])
        else:
            ex = srv = NativeServer(fm, slots=slots, budget_bytes=budget, max_batch_patterns=cap,
                                    check_free_memory=True, packed=not args.serve_bytes, grow=True)
        st = srv.run(w, deadline_s=120.0)
        summ = st.summary()
        summ["offered_patterns_per_s"] = load
        if not args.serve_python:
            summ["arena_bytes"] = srv.arena_bytes
            summ["batches_staged_by_kernels"] = srv.last_run_staged
        # every served count equals one direct count of all patterns of the run
        d_all = fm.count(to_dev(w.pat), to_dev(w.off)).cpu().numpy().view(np.uint32)
        summ["equal_to_direct_count"] = bool(np.array_equal(ex.counts(0, int(w.req_off[-1])), d_all))
        res["loads"].append(summ)
        if not args.serve_python:
            srv.free()
        log("serve load %.0e: p50 %.2f ms p99 %.2f ms, %.2f M patterns/s, %d batches (median %.0f, p99 %.0f patterns; "
            "p99 requests in batches of median %.0f), max in flight %d, equal=%s"
            % (load, summ["p50_ms"], summ["p99_ms"], (summ["patterns_per_s"] or 0) / 1e6, summ["batches"],
               summ.get("batch_patterns_p50", 0), summ.get("batch_patterns_p99", 0),
               summ.get("batch_patterns_of_p99_requests_median", 0), summ["max_inflight_batches"],
               summ["equal_to_direct_count"]))
        del ex, srv
    if not args.serve_python and res["loads"]:
        # a mid load again with the batches copied by hipMemcpyAsync instead of staged by kernels
        mids = [i for i, l in enumerate(res["loads"]) if 1e7 <= l["offered_patterns_per_s"] <= 1e8]
        if mids:
            k = mids[len(mids) // 2]
            load = res["loads"][k]["offered_patterns_per_s"]
            w = make_workload(5000 + k, text, load, args.serve_seconds, max_requests=200_000)
            srv = NativeServer(fm, slots=slots, budget_bytes=budget, max_batch_patterns=cap, check_free_memory=True,
                               packed=not args.serve_bytes, grow=True, copy_engine=True)
            summ = srv.run(w, deadline_s=120.0).summary()
            summ["offered_patterns_per_s"] = load
            d_all = fm.count(to_dev(w.pat), to_dev(w.off)).cpu().numpy().view(np.uint32)
            summ["equal_to_direct_count"] = bool(np.array_equal(srv.counts(0, int(w.req_off[-1])), d_all))
            srv.free()
            res["mid_load_copy_engine"] = summ
            log("serve load %.0e with hipMemcpyAsync batches: p50 %.2f ms p99 %.2f ms, %.2f M patterns/s, equal=%s"
                % (load, summ["p50_ms"], summ["p99_ms"], (summ["patterns_per_s"] or 0) / 1e6,
                   summ["equal_to_direct_count"]))
        # the top load again with the patterns sent the other way (bytes against packed words)
        load = res["loads"][-1]["offered_patterns_per_s"]
        k = len(res["loads"]) - 1
        w = make_workload(5000 + k, text, load, args.serve_seconds, max_requests=200_000)
        srv = NativeServer(fm, slots=slots, budget_bytes=budget, max_batch_patterns=cap, check_free_memory=True,
                           packed=args.serve_bytes, grow=True)
        summ = srv.run(w, deadline_s=120.0).summary()
        summ["offered_patterns_per_s"] = load
        summ["pattern_form"] = "packed" if args.serve_bytes else "bytes"
        d_all = fm.count(to_dev(w.pat), to_dev(w.off)).cpu().numpy().view(np.uint32)
        summ["equal_to_direct_count"] = bool(np.array_equal(srv.counts(0, int(w.req_off[-1])), d_all))
        srv.free()
        res["top_load_other_form"] = summ
        log("serve load %.0e with %s patterns: p50 %.2f ms p99 %.2f ms, %.2f M patterns/s, equal=%s" % (
            load, summ["pattern_form"], summ["p50_ms"], summ["p99_ms"], (summ["patterns_per_s"] or 0) / 1e6,
            summ["equal_to_direct_count"]))
    fm.free()
    return res


def cpu_model():
    """The host CPU as lscpu reports it (model name, family/model/stepping, sockets x cores, L3, and
    the hypervisor when virtualised), falling back to /proc/cpuinfo."""
    import subprocess
    want = ("Model name", "Vendor ID", "CPU family", "Model", "Stepping", "Socket(s)", "Core(s) per socket",
            "Thread(s) per core", "CPU(s)", "L3 cache", "Hypervisor vendor", "CPU max MHz")
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in want and k.strip() not in info:
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if not info.get("Model name"):
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        info["Model name"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return info or None


def host_threads():
    """(threads this process may run on, online CPUs)."""
    try:
        aff = len(os.sched_getaffinity(0))
    except OSError:
        aff = os.cpu_count()
    return aff, os.cpu_count()


def cpu_baseline(packed, n, datagen, np, with_birank=True, fm_inputs=None):
    """The oracle (plain C, OpenMP over queries) on the host cores, on bounded samples of the same
    workloads.  Every oracle call first builds its prefix table over the whole structure (serially),
    which the GPU timing has no counterpart of, so each rate is differential: one call on a sample
    of S queries and one on its first S/4, and the rate is (3/4 S) / (t_S - t_{S/4}); the build
    cancels."""
    import oracle

    def rate(fn, q_all, *rest):
        S = q_all.size
        s = S // 4
        t0 = time.perf_counter()
        fn(q_all[:s], *[r[:s] for r in rest])
        t_small = time.perf_counter() - t0
        t0 = time.perf_counter()
        fn(q_all, *rest)
        t_big = time.perf_counter() - t0
        return (S - s) / max(t_big - t_small, 1e-9), t_small, t_big

    S = 2 * 10 ** 8
    q = datagen.queries(3204, n, S)
    c = datagen.symbols(3205, S)
    r_q, ts, tb = rate(lambda qq, cc: oracle.rank_dna(packed, n, qq, cc), q, c)
    S1 = 2 * 10 ** 7
    cores = oracle.set_threads(1)
    try:
        r_1, ts1, tb1 = rate(lambda qq, cc: oracle.rank_dna(packed, n, qq, cc), q[:S1], c[:S1])
    finally:
        oracle.set_threads(cores)
    del c
    S4 = 10 ** 8
    r_4, ts4, tb4 = rate(lambda qq: oracle.rank4_dna(packed, n, qq), q[:S4])
    del q
    res = {"value": r_q, "unit": "rank queries/s", "cores": cores, "kind": "oracle",
           "sample": "2*10^8 uniform rank(q,c) queries on the same 2^32-base text, timed against its first "
                     "5*10^7 (%.2f s vs %.2f s); the difference removes the oracle's per-call prefix table "
                     "build, as the GPU build is outside the GPU timing" % (tb, ts),
           "one_thread_queries_per_s": r_1,
           "one_thread_sample": "2*10^7 of the same rank(q,c) queries vs their first 5*10^6 on one thread "
                                "(%.2f s vs %.2f s)" % (tb1, ts1),
           "cpu_model": (cpu_model() or {}).get("Model name"),
           "lscpu": cpu_model(),
           "nproc": host_threads()[0],
           "online_cpus": host_threads()[1],
           "rank4_queries_per_s": r_4,
           "rank4_sample": "10^8 uniform rank4 queries vs their first 2.5*10^7 (%.2f s vs %.2f s), same text"
                           % (tb4, ts4)}
    if with_birank:
        nb = 1 << 36
        bits = datagen.bits(3636, nb, 0.5)
        qb = datagen.queries(3736, nb, S)
        r_b, tsb, tbb = rate(lambda qq: oracle.rank_bits(bits, nb, qq), qb)
        res["birank_queries_per_s"] = r_b
        res["birank_sample"] = ("2*10^8 uniform BiRank queries on a 2^36-bit vector of density 0.5 vs their "
                                "first 5*10^7 (%.2f s vs %.2f s)" % (tbb, tsb))
        del bits, qb
    if fm_inputs is not None:
        # FM count: the oracle's suffix-array binary search over the FM row's 2^28-base text (its suffix
        # array from the device input preparation), on the first 3*10^6 of the row's patterns; the
        # search has no per-call table, so this is a plain rate, taken against its first quarter too
        text, sa, pat, off = fm_inputs
        m = off.size - 1
        q = m // 4
        t0 = time.perf_counter()
        oracle.count_sa(text, sa, pat[:int(off[q])], off[:q + 1])
        tq = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.count_sa(text, sa, pat, off)
        tm = time.perf_counter() - t0
        res["fm_count_patterns_per_s"] = (m - q) / max(tm - tq, 1e-9)
        res["fm_count_sample"] = ("the first %d of the FM row's 10^7 patterns (lengths 20..250) on its 2^28-base "
                                  "text by suffix-array binary search, timed against their first quarter "
                                  "(%.2f s vs %.2f s)" % (m, tm, tq))
    return res


if __name__ == "__main__":
    main()
