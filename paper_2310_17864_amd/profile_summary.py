"""Condenses rocprofv3 output into the short text summaries kept under
profiles/ (kernel durations, HBM traffic per dispatch).

    python -m paper_2310_17864_amd.profile_summary stats <dir> <out.txt> --command "..." \
        [--bench-json <bench stdout>]
    python -m paper_2310_17864_amd.profile_summary traffic <fetch_dir> <write_dir> <out.txt> \
        --copy-bytes N --command "..."
    python -m paper_2310_17864_amd.profile_summary counters <dir> <out.txt> --command "..." \
        [--kernel PREFIX]

`stats` reads the kernel_stats.csv of a `--kernel-trace --stats` run and,
given the JSON line the profiled bench.py printed, records the step time the
bench measured itself with HIP events in that same run.
`counters` reads the counter_collection.csv of a `--pmc` run and records,
per kernel, the median per-dispatch value of every counter collected, plus
the ratios the kernel notes use (VALU instructions per active VALU cycle,
wait share of wave cycles, LDS bank conflicts per LDS instruction) and, when
GRBM_GUI_ACTIVE was collected, the shader clock it implies.
`traffic` reads the counter_collection.csv of two `--pmc FETCH_SIZE` /
`--pmc WRITE_SIZE` runs, takes the median per-dispatch value of the
persistent alignment kernel and of the calibration copy kernel (an
elementwise negation of copy_bytes bytes), and records both with the hash of
the kernel sources they were taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["engine.hpp", "internal.hpp", "kernels_common.hpp", "k_batch.hip", "tune.hpp", "api.cpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def stats(d: str, out: str, command: str, top: int = 12, bench_json: str = "") -> None:
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 --kernel-trace --stats summary",
             f"# command: {command}",
             f"# kernel sources: {kernel_source_hash()}"]
    if bench_json:
        import json
        rec = None
        for line in open(bench_json):
            line = line.strip()
            if line.startswith("{"):
                rec = json.loads(line)
        if rec and "ms_per_step" in rec:
            spread = (f" (min {rec['ms_min']:.4f}, max {rec['ms_max']:.4f})"
                      if "ms_min" in rec and "ms_max" in rec else "")
            lines.append(f"# the same run's own step time (HIP events around each graph replay, "
                         f"{rec.get('steps')} steps): ms_per_step = {rec['ms_per_step']:.4f}{spread}")
    lines.append(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_%':>8}  kernel")
    for r in rows[:top]:
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):8.2f}  {r['Name'][:110]}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _per_kernel(path: str, counter: str, pattern: str):
    """{kernel name: (median per-dispatch value, dispatches)} for kernels whose
    name contains `pattern`."""
    vals = {}
    names = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter or pattern not in r["Kernel_Name"]:
            continue
        d = r["Dispatch_Id"]
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
        names[d] = _kname(r["Kernel_Name"])
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {pattern!r} in {path}")
    by = {}
    for d, v in vals.items():
        by.setdefault(names[d], []).append(v)
    return {k: (statistics.median(v), len(v)) for k, v in by.items()}


def traffic(fetch_dir: str, write_dir: str, out: str, copy_bytes: int, command: str,
            kernel: str = "ctca::k_persistent", copy_kernel: str = "elementwise") -> None:
    """One replay of a plan runs each matching kernel once (the pack kernel and
    the critical-chain kernel, concurrently): its traffic is the sum of their
    per-dispatch medians."""
    fpath, wpath = _find(fetch_dir, "counter_collection.csv"), _find(write_dir, "counter_collection.csv")
    fk = _per_kernel(fpath, "FETCH_SIZE", kernel)
    wk = _per_kernel(wpath, "WRITE_SIZE", kernel)
    cf = sum(v for v, _ in _per_kernel(fpath, "FETCH_SIZE", copy_kernel).values())
    cw = sum(v for v, _ in _per_kernel(wpath, "WRITE_SIZE", copy_kernel).values())
    fsum = sum(v for v, _ in fk.values())
    wsum = sum(v for v, _ in wk.values())
    lines = ["# HBM traffic of one launch (per-dispatch medians of the kernels it runs, summed),",
             "# rocprofv3 --pmc, KiB per dispatch, with a plain copy of copy_bytes bytes as the scale",
             f"# command (FETCH_SIZE, then WRITE_SIZE in a second run): {command}",
             f"kernel_source_hash = {kernel_source_hash()}"]
    for k in sorted(fk):
        lines.append(f"# {k}: fetch {fk[k][0]:.1f} KiB, write {wk.get(k, (0, 0))[0]:.1f} KiB "
                     f"({fk[k][1]} dispatches)")
    lines += [f"fetch_kb = {fsum:.1f}", f"write_kb = {wsum:.1f}",
              f"copy_bytes = {copy_bytes}", f"copy_fetch_kb = {cf:.1f}", f"copy_write_kb = {cw:.1f}",
              f"# scaled: read {fsum * copy_bytes / cf / 1e9:.3f} GB, write {wsum * copy_bytes / cw / 1e9:.3f} GB"
              " per replay"]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


XCDS = 8   # accelerator complex dies of an MI355X: GRBM_GUI_ACTIVE counts on each


def _kname(full: str) -> str:
    """A kernel's name without return type, anonymous namespace or arguments
    (template arguments kept)."""
    n = full[5:] if full.startswith("void ") else full
    return n.replace("(anonymous namespace)::", "").split("(")[0]


def counters(d: str, out: str, command: str, kernel: str = "ctca::") -> None:
    path = _find(d, "counter_collection.csv")
    per = {}      # (kernel, counter) -> {dispatch: value}
    dur = {}      # (kernel, dispatch) -> seconds
    for r in csv.DictReader(open(path)):
        if kernel not in r["Kernel_Name"]:
            continue
        k = _kname(r["Kernel_Name"])
        key = (k, r["Counter_Name"])
        disp = per.setdefault(key, {})
        disp[r["Dispatch_Id"]] = disp.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        if r.get("Start_Timestamp") and r.get("End_Timestamp"):
            dur[(k, r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    if not per:
        raise SystemExit(f"no counter rows for kernels matching {kernel!r} in {path}")
    lines = ["# rocprofv3 --pmc summary: per-dispatch medians per kernel",
             f"# command: {command}",
             f"kernel_source_hash = {kernel_source_hash()}"]
    kernels = sorted({k for k, _ in per})
    for k in kernels:
        vals = {c: statistics.median(v.values()) for (kk, c), v in per.items() if kk == k}
        n = max(len(v) for (kk, c), v in per.items() if kk == k)
        lines.append(f"# {k} ({n} dispatches)")
        for c in sorted(vals):
            lines.append(f"{k} {c} = {vals[c]:.6g}")
        def ratio(a, b, label):
            if a in vals and b in vals and vals[b] > 0:
                lines.append(f"{k} {label} = {vals[a] / vals[b]:.4f}")
        ratio("SQ_ACTIVE_INST_VALU", "SQ_INSTS_VALU", "cycles_per_valu_inst")
        ratio("SQ_WAIT_ANY", "SQ_WAVE_CYCLES", "wait_share_of_wave_cycles")
        ratio("SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS", "lds_conflict_cycles_per_lds_inst")
        ratio("SQ_INSTS_VALU", "SQ_WAVES", "valu_insts_per_wave")
        if (k, "GRBM_GUI_ACTIVE") in per:
            # busy GPU cycles per dispatch over its duration: the shader clock
            # (counted on every XCD), and the dispatch's duration under the
            # counter collection (which runs dispatches one at a time)
            g = per[(k, "GRBM_GUI_ACTIVE")]
            clk = [v / dur[(k, i)] / XCDS for i, v in g.items() if dur.get((k, i), 0) > 0]
            if clk:
                lines.append(f"{k} clock_ghz = {statistics.median(clk) / 1e9:.4f}")
                lines.append(f"{k} dispatch_ms_alone = "
                             f"{statistics.median(dur[(k, i)] for i in g if (k, i) in dur) * 1e3:.4f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--bench-json", default="")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    c.add_argument("--kernel", default="ctca::")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("out")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--kernel", default="ctca::k_persistent",
                   help="name prefix of the kernels whose per-dispatch traffic is summed")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        stats(args.dir, args.out, args.command, bench_json=args.bench_json)
    elif args.cmd == "counters":
        counters(args.dir, args.out, args.command, kernel=args.kernel)
    else:
        traffic(args.fetch_dir, args.write_dir, args.out, args.copy_bytes, args.command,
                kernel=args.kernel)


if __name__ == "__main__":
    sys.exit(main())
