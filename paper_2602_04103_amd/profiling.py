"""Summaries of rocprofv3 output for the committed profile records.

  python -m paper_2602_04103_amd.profiling stats DIR [--cmd "..."]        kernel-trace statistics table
  python -m paper_2602_04103_amd.profiling counters DIR COUNTER [...]     per-kernel mean of PMC counters
  python -m paper_2602_04103_amd.profiling traffic FETCH_DIR WRITE_DIR --row ROW --layout 16|32 \
      --form pair|lane|sweep --copy-bytes B --out JSON

`traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) into HBM bytes per launch of the rank
kernel of one benchmark row and layout (the profiled run runs only that row), scaled by what the
same counters read for a plain device copy of known size in the same runs (the calibration
factor).  Entries are merged into JSON under the key "ROW|L<layout>|<form>", each with a hash of the
kernel sources it was taken with; entries whose sources have changed since are dropped."""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the kernel sources each row's counters depend on (a record goes stale when any of them changes)
ROW_SOURCES = {"birank": ["birank.hip", "birank_dev.hpp", "sweep.hpp", "common.hpp"],
               "quadrank": ["quadrank.hip", "quadrank_dev.hpp", "sweep.hpp", "common.hpp"]}
# kernel of each row for each launch form: lane pairs, one lane per query, position-ordered tiles
ROW_KERNELS = {
    "quadrank_rank": {"pair": "qr_rank1_pair_kernel", "lane": "qr_rank1_kernel", "sweep": "qr_sym_sweep_kernel"},
    "quadrank_rank4": {"pair": "qr_rank4_pair_kernel", "lane": "qr_rank4_kernel", "sweep": "qr_rank4_sweep_kernel"},
    "quadrank_prefix_rank": {"pair": "qr_prefix_pair_kernel", "lane": "qr_prefix_kernel", "sweep": "qr_sym_sweep_kernel"},
    "birank_rank_p0.5": {"pair": "br_rank_pair_kernel", "lane": "br_rank_kernel", "sweep": "br_rank_sweep_kernel"},
    "birank_rank_p0.05": {"pair": "br_rank_pair_kernel", "lane": "br_rank_kernel", "sweep": "br_rank_sweep_kernel"},
}


def launch_form(tuning) -> str:
    """'sweep', 'lane' or 'pair': which kernel a row's launch settings select."""
    t = tuning if isinstance(tuning, dict) else {}
    if t.get("sweep"):
        return "sweep"
    return "lane" if t.get("lanes") == 1 else "pair"


# layout name -> the suffix of its trait type in kernel names (qr::BR16P, qr::QR24_8, ...)
LAYOUT_TOKENS = {"16": "16", "32": "32", "16p": "16P", "64": "64", "16x2": "16X2", "24_8": "24_8"}


def traffic_key(row: str, layout, form: str) -> str:
    return "%s|L%s|%s" % (row, layout, form)


def layout_token(row: str, layout) -> str:
    return ("QR" if row.startswith("quadrank") else "BR") + LAYOUT_TOKENS[str(layout)]


def kernel_matches(name: str, row: str, form: str, layout) -> bool:
    """Whether a (demangled) kernel name from a profile is the given row's kernel in that form and
    layout.  rank and prefix_rank share the sweep kernel; its PREFIX argument tells them apart."""
    import re
    fam = ROW_KERNELS[row][form]
    if fam + "<" not in name or not re.search(r"\b%s\b" % re.escape(layout_token(row, layout)), name):
        return False
    if fam == "qr_sym_sweep_kernel":
        return (", true," in name) == (row == "quadrank_prefix_rank")
    return True


def _csvs(d: str, suffix: str):
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _rows(path: str):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def kernel_stats(d: str):
    out = []
    for p in _csvs(d, "kernel_stats.csv"):
        out += _rows(p)
    return out


def counter_values(d: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    res = {}
    for p in _csvs(d, "counter_collection.csv"):
        for r in _rows(p):
            name = r.get("Counter_Name") or r.get("Counter-Name")
            if name != counter:
                continue
            k = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
            res.setdefault(k, []).append(float(r.get("Counter_Value") or r.get("Counter-Value") or 0))
    return res


def counter_dispatches(d: str, counter: str):
    """{kernel name: [(dispatch id, value)] in dispatch order} for one counter."""
    res = {}
    for p in _csvs(d, "counter_collection.csv"):
        for r in _rows(p):
            name = r.get("Counter_Name") or r.get("Counter-Name")
            if name != counter:
                continue
            k = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
            did = int(r.get("Dispatch_Id") or r.get("Dispatch-Id") or r.get("Correlation_Id") or 0)
            res.setdefault(k, []).append((did, float(r.get("Counter_Value") or r.get("Counter-Value") or 0)))
    for v in res.values():
        v.sort()
    return res


def source_hash(names) -> str:
    h = hashlib.sha256()
    for nme in names:
        with open(os.path.join(ROOT, "paper_2602_04103_amd", "csrc", nme), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _match(kernels: dict, needle: str):
    vals = []
    for k, v in kernels.items():
        if needle in k:
            vals += v
    return vals


def cmd_stats(a):
    rows = kernel_stats(a.dir)
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0) or 0))
    print("# rocprofv3 --kernel-trace --stats summary")
    if a.cmd:
        print("# command: " + a.cmd)
    print("%-90s %8s %14s %12s %7s" % ("kernel", "calls", "total_ns", "avg_ns", "pct"))
    for r in rows:
        print("%-90s %8s %14s %12.0f %7.2f" % (r["Name"][:90], r["Calls"], r["TotalDurationNs"],
                                               float(r["AverageNs"]), float(r.get("Percentage", 0) or 0)))


def cmd_counters(a):
    print("# rocprofv3 --pmc per-kernel mean over dispatches")
    if a.cmd:
        print("# command: " + a.cmd)
    for c in a.counter:
        vals = counter_values(a.dir, c)
        for k, v in sorted(vals.items()):
            print("%-24s %-80s dispatches=%-5d mean=%.4g" % (c, k[:80], len(v), statistics.mean(v)))


def cmd_dispatches(a):
    """Each dispatch's counter value, in dispatch order, for the kernels whose names contain a given
    text: for runs that launch one kernel on several inputs in turn (the bench's gather sweep)."""
    print("# rocprofv3 --pmc per-dispatch values, in dispatch order")
    if a.cmd:
        print("# command: " + a.cmd)
    for c in a.counter:
        for k, v in sorted(counter_dispatches(a.dir, c).items()):
            if a.kernel and a.kernel not in k:
                continue
            print("%-24s %s" % (c, k[:100]))
            print("    " + " ".join("%.4g" % x for _, x in v))


def cmd_traffic(a):
    fetch = counter_values(a.fetch_dir, "FETCH_SIZE")
    write = counter_values(a.write_dir, "WRITE_SIZE")
    copy_f = _match(fetch, a.copy_kernel)
    copy_w = _match(write, a.copy_kernel)
    if not copy_f or not copy_w:
        sys.exit("no calibration copy kernel '%s' in the counter output" % a.copy_kernel)
    # the copy reads and writes copy_bytes once each: factors convert counter KiB to bytes
    f_fac = a.copy_bytes / (max(copy_f) * 1024.0)
    w_fac = a.copy_bytes / (max(copy_w) * 1024.0)
    out = {"kernels": {}}
    try:
        with open(a.out) as f:
            prev = json.load(f)
        for k, v in prev.get("kernels", {}).items():  # keep records whose sources are unchanged
            if v.get("source_hash") == source_hash(v.get("sources", [])):
                out["kernels"][k] = v
    except (OSError, ValueError):
        pass
    srcs = ROW_SOURCES["quadrank" if a.row.startswith("quadrank") else "birank"]
    token = layout_token(a.row, a.layout)
    sel = lambda d: [x for k, v in d.items() if kernel_matches(k, a.row, a.form, a.layout) for x in v]  # noqa: E731
    fv, wv = sel(fetch), sel(write)
    kname = ROW_KERNELS[a.row][a.form]
    if not fv or not wv:
        sys.exit("no dispatches of %s for layout %s in the counter output" % (kname, a.layout))
    out["kernels"][traffic_key(a.row, a.layout, a.form)] = {
        "kernel": "%s<%s>" % (kname, token),
        "sources": srcs,
        "source_hash": source_hash(srcs),
        "dispatches": len(fv),
        "fetch_kib_per_dispatch": statistics.mean(fv),
        "write_kib_per_dispatch": statistics.mean(wv),
        "fetch_factor": f_fac,
        "write_factor": w_fac,
        "copy_bytes": a.copy_bytes,
        "hbm_bytes_per_launch": statistics.mean(fv) * 1024.0 * f_fac + statistics.mean(wv) * 1024.0 * w_fac,
    }
    if a.cmd:
        out["kernels"][traffic_key(a.row, a.layout, a.form)]["command"] = a.cmd
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", default="")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("counter", nargs="+")
    c.add_argument("--cmd", default="")
    dsp = sub.add_parser("dispatches")
    dsp.add_argument("dir")
    dsp.add_argument("counter", nargs="+")
    dsp.add_argument("--kernel", default="", help="only kernels whose name contains this text")
    dsp.add_argument("--cmd", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--row", required=True, choices=sorted(ROW_KERNELS))
    t.add_argument("--layout", required=True, choices=tuple(LAYOUT_TOKENS))
    t.add_argument("--form", default="pair", choices=("pair", "lane", "sweep"),
                   help="launch form the profiled run used (its tuning)")
    t.add_argument("--cmd", default="", help="the profiled command, stored with the record")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--copy-kernel", default="elementwise")
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    {"stats": cmd_stats, "counters": cmd_counters, "dispatches": cmd_dispatches, "traffic": cmd_traffic}[a.what](a)


if __name__ == "__main__":
    main()
