"""Host-side behaviour of bench.py: the one-GPU guard and the counter summary
that supplies the roofline's measured traffic (valid only while the kernel's
source is the one the counters were taken on)."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    with open(bench.COUNTERS) as f:
        summ = json.load(f)
    ent = summ["kernels"]["graph_spmm"]
    got = bench.measured_traffic("graph_spmm")
    assert got == pytest.approx((ent["fetch_kib_per_launch"] * summ["fetch_factor"] +
                                 ent["write_kib_per_launch"] * summ["write_factor"]) * 1024.0)
    assert bench.measured_traffic("no_such_kernel") is None
    # a summary taken on another version of the source gives no traffic
    summ["kernels"]["graph_spmm"]["source_sha256"] = "0" * 64
    alt = tmp_path / "counters.json"
    alt.write_text(json.dumps(summ))
    monkeypatch.setattr(bench, "COUNTERS", str(alt))
    assert bench.measured_traffic("graph_spmm") is None


def test_gather_model_bytes():
    """The roofline's per-launch bytes follow the gather model
    8 (n + 1) + 8 nnz + e k nnz + 2 e n k for both sparse x dense products."""
    info = dict(n=10, nnz_M=100, kp=6, arcs=40, d=4, pairs=0, es=4, nnz_counts=0)
    assert bench.kernel_bytes("spmm", info) == 88 + 800 + 4 * 6 * 100 + 2 * 4 * 10 * 6
    assert bench.kernel_bytes("graph_spmm", info) == 88 + 320 + 4 * 4 * 40 + 2 * 4 * 10 * 4
    # the Chebyshev recurrence of order 10: 21 launches moving 80 dense streams
    assert bench.graph_spmm_streams(10) == (21, 80)
    assert bench.graph_spmm_streams(1) == (3, 8)


def _write_csv(path, header, rows):
    import csv
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_rocprof_summaries(tmp_path):
    """The committed summariser turns rocprofv3 csv output into the profile
    tables and the counter JSON that measured_traffic reads."""
    kt = tmp_path / "kt" / "host" / "123_kernel_stats.csv"
    _write_csv(kt, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [["void lne::(anonymous namespace)::k_graph_spmm<32, false, 8, true, false, "
                 "float>(long const*, int const*)", 42, 42 * 30e6, 30e6, 60.0],
                ["k_hist", 12, 12 * 7e6, 7e6, 10.0]])
    md = bench.summarize_kernel_trace(str(tmp_path / "kt"), 2, "T", "cmd")
    assert "`k_graph_spmm<32, false, 8, true, false, float>` | 42 | 30.000 | 630.0 |" in md
    assert "`k_hist` | 12 | 7.000 | 42.0 |" in md
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write_csv(tmp_path / "f" / "h" / "1_counter_collection.csv", hdr,
               [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0],
                [5, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 511.0],
                [6, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 513.0],
                [9, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 9999.0],
                [2, "void k_graph_spmm<32, false, 8, true, false, float>()", "FETCH_SIZE", 100.0],
                [3, "void k_graph_spmm<32, false, 8, true, false, float>()", "FETCH_SIZE", 300.0],
                [4, "void k_spmm<32, true, 8, true, float, float, float>()", "FETCH_SIZE", 7.0]])
    _write_csv(tmp_path / "w" / "h" / "1_counter_collection.csv", hdr,
               [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0],
                [5, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0],
                [6, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0],
                [9, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 4096.0],
                [2, "void k_graph_spmm<32, false, 8, true, false, float>()", "WRITE_SIZE", 10.0],
                [3, "void k_graph_spmm<32, false, 8, true, false, float>()", "WRITE_SIZE", 30.0]])
    summ = bench.summarize_counters(str(tmp_path / "f"), str(tmp_path / "w"), 1 << 20, "x", ["c"])
    assert summ["fetch_factor"] == pytest.approx(2.0)
    assert summ["write_factor"] == pytest.approx(1.0)
    gs = summ["kernels"]["graph_spmm"]
    assert gs["launches"] == 2 and gs["fetch_kib_per_launch"] == 200.0
    assert gs["write_kib_per_launch"] == 20.0 and len(gs["source_sha256"]) == 64
    assert summ["kernels"]["spmm"]["fetch_kib_per_launch"] == 7.0
    assert "graph_spmm" in bench.counters_markdown(summ, "t")
