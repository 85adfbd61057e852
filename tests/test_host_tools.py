"""Host logic without a GPU: the measurement tools and the benchmark's
argument contract.

* rocprof_summary pmc: HBM bytes per launch = FETCH_SIZE * 1024 * (1 GiB /
  the multiply's FETCH_SIZE) + WRITE_SIZE * 1024 * (1 GiB / the fill's
  WRITE_SIZE), averaged over the selected dispatches (the last N before the
  skipped last M).
* rocprof_summary stats: the last-N average of a kernel from the
  per-dispatch trace.
* rocprof_summary mfma: flops, time and utilisation from the counters, over
  the dispatches between two markers.
* bench.py --gpus 2 exits with status 2 and says why, before touching a GPU.
"""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1606_01273_amd import rocprof_summary as rs  # noqa: E402

KIB = 1024.0
GIB = float(1 << 30)


def _write_counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_pmc_traffic_scaling_and_dispatch_selection(tmp_path):
    # fill writes 1 GiB and the counter reads exactly that; the multiply's
    # fetch counter reads half of 1 GiB (scale 2)
    fetch = [(1, "k_residual_rows", "FETCH_SIZE", 9e9),           # a trial launch (not selected)
             (2, "k_residual_rows", "FETCH_SIZE", 1000.0),
             (3, "k_residual_rows", "FETCH_SIZE", 3000.0),
             (4, "k_residual_rows", "FETCH_SIZE", 7e9),           # a later pass (skipped)
             (5, "MulFunctor", "FETCH_SIZE", GIB / KIB / 2)]
    write = [(1, "k_residual_rows", "WRITE_SIZE", 9e9),
             (2, "k_residual_rows", "WRITE_SIZE", 500.0),
             (3, "k_residual_rows", "WRITE_SIZE", 1500.0),
             (4, "k_residual_rows", "WRITE_SIZE", 7e9),
             (5, "FillFunctor", "WRITE_SIZE", GIB / KIB)]
    fc, wc = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    _write_counters(fc, fetch)
    _write_counters(wc, write)
    out_json, out_txt = str(tmp_path / "t.json"), str(tmp_path / "t.txt")
    sys.argv = ["rs", "pmc", fc, wc, out_json, out_txt, "--key", "k/A/e", "--kernel", "residual_rows",
                "--last", "2", "--skip-last", "1", "--command-fetch", "cf", "--command-write", "cw"]
    rs.main()
    rec = json.load(open(out_json))["k/A/e"]
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["dispatches"] == [2, 2]
    assert rec["bytes_per_launch"] == pytest.approx(2000.0 * KIB * 2.0 + 1000.0 * KIB * 1.0)


def test_stats_last_dispatch_average(tmp_path):
    stats = str(tmp_path / "s.csv")
    with open(stats, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs"])
        w.writerow(["k_residual_rows", 5, 5000, 1000])
    trace = str(tmp_path / "t.csv")
    with open(trace, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for d, dur in enumerate([9000, 1000, 3000, 7000, 7000]):
            w.writerow([d, "k_residual_rows", 100 * d, 100 * d + dur])
    out = str(tmp_path / "o.txt")
    sys.argv = ["rs", "stats", stats, out, "--command", "c", "--trace", trace, "--last-kernel", "residual_rows",
                "--last", "2", "--skip-last", "2"]
    rs.main()
    text = open(out).read()
    assert "average 2.00 us" in text           # (1000 + 3000) / 2 ns
    assert "skipped last 2 dispatches" in text and "average 7.00 us" in text


def test_mfma_counters_between_markers(tmp_path):
    rows = []
    # marker kernel dispatches 1, 10, 20; GEMM dispatches 5 (trial), 12 and 22
    rows += [(1, "k_residual_rows", "GRBM_GUI_ACTIVE", 8.0)]
    rows += [(5, "k_gemm", "SQ_INSTS_VALU_MFMA_MOPS_F64", 1e9), (5, "k_gemm", "SQ_VALU_MFMA_BUSY_CYCLES", 1.0),
             (5, "k_gemm", "GRBM_GUI_ACTIVE", 8.0)]
    rows += [(10, "k_residual_rows", "GRBM_GUI_ACTIVE", 8.0)]
    # 2.4e6 active cycles summed over the 8 XCDs: 2.4e6 / (8 * 2.4 GHz) = 125 us
    rows += [(12, "k_gemm", "SQ_INSTS_VALU_MFMA_MOPS_F64", 1e7), (12, "k_gemm", "SQ_VALU_MFMA_BUSY_CYCLES", 1.536e8),
             (12, "k_gemm", "GRBM_GUI_ACTIVE", 2.4e6)]
    rows += [(20, "k_residual_rows", "GRBM_GUI_ACTIVE", 8.0)]
    rows += [(22, "k_gemm", "SQ_INSTS_VALU_MFMA_MOPS_F64", 1e9), (22, "k_gemm", "SQ_VALU_MFMA_BUSY_CYCLES", 1.0),
             (22, "k_gemm", "GRBM_GUI_ACTIVE", 8.0)]
    path = str(tmp_path / "m.csv")
    _write_counters(path, rows)
    out = str(tmp_path / "m.txt")
    sys.argv = ["rs", "mfma", path, out, "--command", "c", "--from-last", "residual_rows", "2", "--before-last", "1"]
    rs.main()
    line = [ln for ln in open(out).read().splitlines() if ln.rstrip().endswith("k_gemm")][0].split()
    # one dispatch; 512 * 1e7 flop = 5.12 GFLOP; time 2.4e6 / (8 * 2.4e9) s = 125 us; 40.96 TF/s;
    # utilisation 1.536e8 / (2.4e6 / 8 * 1024) = 50 %
    assert line[0] == "1"
    assert float(line[1]) == pytest.approx(5.12, rel=1e-3)
    assert float(line[4]) == pytest.approx(125.0, rel=1e-3)
    assert float(line[5]) == pytest.approx(40.96, rel=1e-3)
    assert line[6] == "50.0%"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
