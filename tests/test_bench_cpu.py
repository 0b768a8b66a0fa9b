"""Host-side checks of bench.py (no GPU): the one-GPU rule, the paper's FLOP
accounting, and the guard that keeps stale byte counters out of the JSON line."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_paper_flops_counts_2n3_per_product():
    """Sec. V-B: 2 n^3 per n x n x n product; Newton-Schulz has two per iteration,
    the third-order step three; restarted (FP32) iterations count as well."""
    st = {"n": np.array([10, 20]), "iters_lo": np.array([3, 1]), "iters_fb": np.array([1, 0])}
    assert bench.paper_flops(st) == 2 * 2 * (1000 * 4 + 8000 * 1)
    assert bench.paper_flops(st, products_per_iter=3) == 2 * 3 * (1000 * 4 + 8000 * 1)


def test_traffic_profile_is_used_only_for_its_kernel_workload_and_schedule(tmp_path,
                                                                           monkeypatch):
    with open(bench.TRAFFIC_PATH) as fh:
        rec = json.load(fh)
    fake = dict(rec, kernel_sources_sha256=bench.kernel_sources_sha256(), per_launch_bytes=123.0)
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(fake))
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(path))
    assert bench.measured_traffic(fake["workload"], fake["schedule"]) == 123.0
    assert bench.measured_traffic(fake["workload"], "other schedule") is None
    assert bench.measured_traffic("other workload", fake["schedule"]) is None
    path.write_text(json.dumps(dict(fake, kernel_sources_sha256="0" * 64)))
    assert bench.measured_traffic(fake["workload"], fake["schedule"]) is None


def test_committed_traffic_profile_is_complete():
    """The committed byte-counter summary names its kernel sources, workload,
    schedule, calibration and command (bench.py uses it only when all match)."""
    with open(bench.TRAFFIC_PATH) as fh:
        rec = json.load(fh)
    assert len(rec["kernel_sources_sha256"]) == 64
    assert rec["workload"] and rec["schedule"] and rec["command"].startswith("rocprofv3 --pmc")
    assert rec["calibration"]["fetch_scale"] > 0 and rec["calibration"]["write_scale"] > 0
    # one launch = the mean of a SQUARE and an UPDATE launch, reads plus writes
    both = sum(rec[k]["fetch_bytes"] + rec[k]["write_bytes"] for k in ("square", "update"))
    assert rec["per_launch_bytes"] == pytest.approx(both / 2, rel=1e-9)
