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
