"""bench.py's derived figures, checked without a GPU: the roofline arithmetic, the traffic
record being used only for the workload, launch count and kernel sources it was taken on, and
the one-GPU refusal."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_arithmetic():
    r = bench.roofline(8.0e9, 2.0, 4, "k")
    assert r["achieved"] == pytest.approx(4000.0)          # 8 GB in 2 ms
    assert r["frac"] == pytest.approx(0.5)
    assert r["peak"] == bench.HBM_PEAK_GBS == 8000.0
    assert r["avg_launch_us"] == pytest.approx(500.0)
    assert r["traffic"] is None and r["bound"] == "hbm" and r["unit"] == "GB/s"


def test_traffic_record_is_tied_to_its_sources():
    path = os.path.join(ROOT, "profiles", "lm0_traffic.json")
    rec = json.load(open(path))
    per_launch = (rec["fetch_bytes"] + rec["write_bytes"]) / rec["launches"]
    if rec["sources_sha256"] == bench.kernel_sources_sha():
        assert bench.measured_traffic(rec["workload"], rec["launches"]) == pytest.approx(per_launch)
    else:
        assert bench.measured_traffic(rec["workload"], rec["launches"]) is None
    assert bench.measured_traffic("another_workload", rec["launches"]) is None
    assert bench.measured_traffic(rec["workload"], rec["launches"] + 1) is None
    # the calibration a 1 GiB copy gives: FETCH_SIZE reads half the bytes, WRITE_SIZE all
    assert rec["calibration"]["fetch_factor"] == pytest.approx(2.0, rel=1e-3)
    assert rec["calibration"]["write_factor"] == pytest.approx(1.0, rel=1e-3)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""
