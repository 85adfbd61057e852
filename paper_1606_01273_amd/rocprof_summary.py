"""Summaries of rocprofv3 output for the measurement record (text and JSON).

  python -m paper_1606_01273_amd.rocprof_summary stats KERNEL_STATS_CSV OUT_TXT --command CMD \
      [--trace KERNEL_TRACE_CSV --last-kernel REGEX --last N]
  python -m paper_1606_01273_amd.rocprof_summary pmc FETCH_CSV WRITE_CSV OUT_JSON OUT_TXT \
      --key WORKLOAD/READING/ENTRY --kernel REGEX --command-fetch CMD --command-write CMD
  python -m paper_1606_01273_amd.rocprof_summary mfma COUNTER_CSV OUT_TXT --command CMD

The PMC form reads two counter-collection CSVs (one run with FETCH_SIZE, one
with WRITE_SIZE, both in KiB per dispatch) and scales them with the same
counters read for calibration kernels of known traffic run in the same
process (a fill of 1 GiB: writes 1 GiB; an element-wise multiply of 1 GiB:
reads 1 GiB and writes 1 GiB).  The HBM bytes per launch of the matched
kernel are fetch * 1024 * fetch_scale + write * 1024 * write_scale.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys

GIB = float(1 << 30)
HERE = os.path.dirname(os.path.abspath(__file__))


def rows_kernel_source_sha256() -> str:
    """Hash of the source text of the streaming residual kernel (the region
    from its template line to the separable-energy helper in kernels.hip): a
    recorded traffic figure is valid only for this exact kernel source."""
    path = os.path.join(HERE, "csrc", "kernels.hip")
    with open(path) as fh:
        src = fh.read()
    a = src.index("template <typename T, int NST>\n__global__ __launch_bounds__(256) void k_residual_rows(")
    b = src.index("// separable row energies from the full table")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def _per_dispatch(path: str, counter: str):
    """counter value per dispatch, per kernel name, in dispatch order"""
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r.get("Counter_Name") != counter:
                continue
            rows.append((int(r.get("Dispatch_Id") or 0), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort(key=lambda t: t[0])
    out = {}
    for _, name, v in rows:
        out.setdefault(name, []).append(v)
    return out


def cmd_stats(a):
    with open(a.csv) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel-trace statistics", f"# command: {a.command}", "",
             f"{'total ms':>10} {'calls':>7} {'avg us':>10} {'%':>6}  kernel"]
    for r in rows[: a.top]:
        name = re.sub(r"\s+", " ", r["Name"])[:110]
        lines.append(f"{float(r['TotalDurationNs']) / 1e6:10.3f} {int(r['Calls']):7d} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {100 * float(r['TotalDurationNs']) / tot:6.2f}  {name}")
    if a.trace and a.last_kernel and a.last > 0:
        # per-dispatch durations of one kernel from the kernel trace: the last
        # N dispatches are the timed ones (earlier ones include the
        # autotuner's trial launches of other launch shapes)
        kre = re.compile(a.last_kernel)
        disp = []
        with open(a.trace) as fh:
            for r in csv.DictReader(fh):
                if kre.search(r.get("Kernel_Name", "")):
                    disp.append((int(r.get("Dispatch_Id") or 0),
                                 int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        disp.sort()
        tail = [d for _, d in disp[-a.skip_last:]] if a.skip_last > 0 else []
        if a.skip_last > 0:
            disp = disp[:-a.skip_last]
        sel = [d for _, d in disp[-a.last:]]
        if sel:
            skip = f", skipping the last {a.skip_last}" if a.skip_last > 0 else ""
            lines += ["", f"last {len(sel)} dispatches of {a.last_kernel}{skip} (of {len(disp) + a.skip_last}): "
                          f"average {sum(sel) / len(sel) / 1e3:.2f} us, min {min(sel) / 1e3:.2f} us, "
                          f"max {max(sel) / 1e3:.2f} us"]
        if tail:
            lines += [f"the skipped last {len(tail)} dispatches (a later pass of the command): average "
                      f"{sum(tail) / len(tail) / 1e3:.2f} us, min {min(tail) / 1e3:.2f} us, max {max(tail) / 1e3:.2f} us"]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines[:12] + lines[-2:]))


def cmd_pmc(a):
    fetch = _per_dispatch(a.fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(a.write_csv, "WRITE_SIZE")
    kre = re.compile(a.kernel)

    def pick(d, pat):
        vals = [v for k, vs in d.items() if re.search(pat, k) for v in vs]
        return vals

    kf, kw = pick(fetch, kre), pick(write, kre)
    if not kf or not kw:
        sys.exit(f"no dispatch of {a.kernel} in the counter files")
    if a.skip_last > 0:   # launches after the ones wanted (a later pass of the same command)
        kf, kw = kf[:-a.skip_last], kw[:-a.skip_last]
    if a.last > 0:   # the timed launches only (not the autotuner's trial launches before them)
        kf, kw = kf[-a.last:], kw[-a.last:]
    fill_w = pick(write, r"FillFunctor")
    mul_f = pick(fetch, r"MulFunctor")
    mul_w = pick(write, r"MulFunctor")
    # calibration dispatches: the ones moving about 1 GiB
    fill_w = [v for v in fill_w if v * 1024 > 0.5 * GIB]
    mul_f = [v for v in mul_f if v * 1024 > 0.25 * GIB]
    mul_w = [v for v in mul_w if v * 1024 > 0.5 * GIB]
    if not fill_w or not mul_f:
        sys.exit("calibration dispatches not found (run the bench with --copy-calibration)")
    fetch_scale = GIB / (1024 * mul_f[-1])
    write_scale = GIB / (1024 * fill_w[-1])
    f_kib = sum(kf) / len(kf)
    w_kib = sum(kw) / len(kw)
    traffic = f_kib * 1024 * fetch_scale + w_kib * 1024 * write_scale
    rec = {"bytes_per_launch": traffic, "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
           "dispatches": [len(kf), len(kw)], "fetch_scale": fetch_scale, "write_scale": write_scale,
           "calibration": {"fill_write_kib": fill_w[-1], "mul_fetch_kib": mul_f[-1],
                           "mul_write_kib": mul_w[-1] if mul_w else None},
           "kernel_regex": a.kernel, "last_dispatches": a.last, "skipped_last": a.skip_last,
           "kernel_source_sha256": rows_kernel_source_sha256(),
           "command_fetch": a.command_fetch, "command_write": a.command_write}
    db = {}
    if os.path.exists(a.out_json):
        with open(a.out_json) as fh:
            db = json.load(fh)
    db[a.key] = rec
    with open(a.out_json, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    lines = [f"# rocprofv3 PMC traffic of {a.kernel} ({a.key})",
             f"# FETCH_SIZE run: {a.command_fetch}", f"# WRITE_SIZE run: {a.command_write}", "",
             f"dispatches (fetch, write): {len(kf)}, {len(kw)}",
             f"FETCH_SIZE per dispatch: {f_kib:.1f} KiB   WRITE_SIZE per dispatch: {w_kib:.1f} KiB",
             f"calibration: fill of 1 GiB -> WRITE_SIZE {fill_w[-1]:.1f} KiB (scale {write_scale:.4f}); "
             f"multiply of 1 GiB -> FETCH_SIZE {mul_f[-1]:.1f} KiB (scale {fetch_scale:.4f})",
             f"HBM bytes per launch: {traffic / 1e9:.4f} GB"]
    with open(a.out_txt, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_mfma(a):
    """Per kernel: the F64 MFMA work (SQ_INSTS_VALU_MFMA_MOPS_F64, units of 512
    flops), the MFMA busy cycles and the GPU-active cycles of the dispatch
    (averages per dispatch).  The dispatch time is the GPU-active count (summed
    over the XCDs) over the XCD count and the clock; utilisation is the busy
    count (per SIMD) over the GPU-active cycles of every SIMD."""
    per = {}
    with open(a.csv) as fh:
        for r in csv.DictReader(fh):
            key = (r["Kernel_Name"], int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0))
            per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    first, stop = 0, None
    if a.from_last:
        # keep the dispatches from the N-th last dispatch of the marker kernel
        # on (the timed region; earlier ones include the autotuner's trials),
        # and, with --before-last M, before its M-th last (a later pass)
        mre, n = re.compile(a.from_last[0]), int(a.from_last[1])
        ids = sorted(d for (name, d) in per if mre.search(name))
        if len(ids) >= n:
            first = ids[-n]
        if a.before_last and len(ids) >= a.before_last:
            stop = ids[-a.before_last]
    agg = {}
    for (name, did), c in per.items():
        if did < first or (stop is not None and did >= stop):
            continue
        short = re.sub(r"\(.*", "", re.sub(r"\s+", " ", name))[:70]
        g = agg.setdefault(short, {"n": 0, "busy": 0.0, "gui": 0.0, "mops": 0.0})
        g["n"] += 1
        g["busy"] += c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        g["gui"] += c.get("GRBM_GUI_ACTIVE", 0.0)
        g["mops"] += c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
    lines = [f"# rocprofv3 MFMA counters per kernel (averages per dispatch)", f"# command: {a.command}",
             (f"# dispatches from the {a.from_last[1]}-th last of {a.from_last[0]} on"
              + (f", before its {a.before_last}-th last" if a.before_last else "")) if a.from_last else "#",
             "# F64 MFMA GFLOP = 512 * SQ_INSTS_VALU_MFMA_MOPS_F64 / 1e9; GRBM_GUI_ACTIVE is summed over the",
             f"# {a.xcds} XCDs, so the dispatch time is GUI_ACTIVE / ({a.xcds} * {a.clock_ghz} GHz); MFMA_BUSY counts per",
             f"# SIMD: utilisation = MFMA_BUSY / (GUI_ACTIVE / {a.xcds} * {a.simds} SIMDs)", "",
             f"{'dispatches':>10} {'F64 GFLOP':>10} {'MFMA_BUSY':>14} {'GUI_ACTIVE':>12} {'time us':>9} "
             f"{'TF/s':>7} {'MFMA util':>9}  kernel"]
    for k, g in sorted(agg.items(), key=lambda kv: -kv[1]["mops"]):
        n = g["n"]
        gf = 512 * g["mops"] / n / 1e9
        t = g["gui"] / n / (a.xcds * a.clock_ghz * 1e9)
        util = g["busy"] / (g["gui"] / a.xcds * a.simds) if g["gui"] > 0 else float("nan")
        lines.append(f"{n:10d} {gf:10.3f} {g['busy'] / n:14.0f} {g['gui'] / n:12.0f} {t * 1e6:9.1f} "
                     f"{gf / 1e3 / t if t > 0 else 0:7.2f} {100 * util:8.1f}%  {k}")
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_pmcsum(a):
    """HBM bytes of every kernel matching a regex, per residual evaluation of
    one state: the counters of all its dispatches in the run (each scaled by
    the calibration factors) divided by the number of evaluations the run
    made, next to the algorithmic bytes of one evaluation."""
    fetch = _per_dispatch(a.fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(a.write_csv, "WRITE_SIZE")
    fill_w = [v for k, vs in write.items() if re.search(r"FillFunctor", k) for v in vs if v * 1024 > 0.5 * GIB]
    mul_f = [v for k, vs in fetch.items() if re.search(r"MulFunctor", k) for v in vs if v * 1024 > 0.25 * GIB]
    if not fill_w or not mul_f:
        sys.exit("no calibration dispatches (fill / multiply of 1 GiB) in the counter files")
    wscale = GIB / (fill_w[-1] * 1024)
    fscale = GIB / (mul_f[-1] * 1024)
    kre = re.compile(a.kernel)
    rows = []
    for name in sorted(set(fetch) | set(write)):
        if not kre.search(name) or re.search(r"Functor", name):
            continue
        nf, nw = fetch.get(name, []), write.get(name, [])
        by = (sum(nf) * fscale + sum(nw) * wscale) * 1024 / a.evals
        rows.append((by, max(len(nf), len(nw)) / a.evals, re.sub(r"\s+", " ", name)[:100]))
    rows.sort(key=lambda r: -r[0])
    tot = sum(r[0] for r in rows)
    lines = ["# rocprofv3 PMC traffic per residual evaluation of one state",
             f"# FETCH_SIZE run: {a.command_fetch}", f"# WRITE_SIZE run: {a.command_write}", "",
             f"evaluations in the run: {a.evals}; calibration scales: fetch {fscale:.4f}, write {wscale:.4f}",
             f"algorithmic bytes of one evaluation (read x and the source, write sigma): {a.algo_bytes / 1e9:.3f} GB",
             "", f"{'GB/eval':>9} {'disp/eval':>9}  kernel"]
    for by, n, name in rows:
        lines.append(f"{by / 1e9:9.3f} {n:9.1f}  {name}")
    lines += ["", f"total of the matched kernels: {tot / 1e9:.3f} GB per evaluation = "
                  f"{tot / a.algo_bytes:.2f} x the algorithmic bytes"]
    with open(a.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--trace", help="kernel trace CSV (per-dispatch timestamps)")
    s.add_argument("--last-kernel", help="kernel regex for the last-N average")
    s.add_argument("--last", type=int, default=0)
    s.add_argument("--skip-last", type=int, default=0, help="ignore the last M dispatches of that kernel")
    p = sub.add_parser("pmc")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("out_json")
    p.add_argument("out_txt")
    p.add_argument("--key", required=True)
    p.add_argument("--kernel", required=True)
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    p.add_argument("--last", type=int, default=0, help="average over the last N dispatches of the kernel only")
    p.add_argument("--skip-last", type=int, default=0, help="ignore the last M dispatches of the kernel")
    m = sub.add_parser("mfma")
    m.add_argument("csv")
    m.add_argument("out")
    m.add_argument("--command", required=True)
    m.add_argument("--xcds", type=int, default=8)
    m.add_argument("--simds", type=int, default=1024)
    m.add_argument("--clock-ghz", type=float, default=2.4)
    m.add_argument("--from-last", nargs=2, metavar=("KERNEL_REGEX", "N"),
                   help="only dispatches from the N-th last dispatch of this kernel on")
    m.add_argument("--before-last", type=int, default=0,
                   help="with --from-last: only dispatches before the M-th last dispatch of that kernel")
    q = sub.add_parser("pmcsum")
    q.add_argument("fetch_csv")
    q.add_argument("write_csv")
    q.add_argument("out")
    q.add_argument("--kernel", required=True)
    q.add_argument("--evals", type=int, required=True, help="residual evaluations of one state in the run")
    q.add_argument("--algo-bytes", type=float, required=True)
    q.add_argument("--command-fetch", required=True)
    q.add_argument("--command-write", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "pmc": cmd_pmc, "mfma": cmd_mfma, "pmcsum": cmd_pmcsum}[a.cmd](a)


if __name__ == "__main__":
    main()
