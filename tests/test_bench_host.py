"""Host-side parts of the benchmark: the one-GPU rule, the stored counter
readings' validity, and the first-come-first-served queue of the served
stream's one-at-a-time comparison."""
import json
import os
import subprocess
import sys

import pytest

from paper_2503_19925_amd import build
from paper_2503_19925_amd.serve import fcfs_latencies

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_is_used_only_for_its_build():
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    want = rec["workloads"]["solve_512"]["k_back_update"]["hbm_bytes_per_launch"]
    if rec["kernel_build_id"] == build.build_id():
        assert bench.measured_traffic("solve_512", "k_back_update") == want
    other = dict(build.tuned_knobs(), EXACT_LINE_BATCH=2)
    assert build.build_id(other) != rec["kernel_build_id"]
    assert bench.measured_traffic("no_such_workload", "k_back_update") is None


def test_fcfs_queue_worked_example():
    # arrivals 0, 1, 1.5, 10; service 2, 2, 1, 1: finishes 2, 4, 5, 11
    lat, last = fcfs_latencies([0.0, 1.0, 1.5, 10.0], [2.0, 2.0, 1.0, 1.0])
    assert lat == pytest.approx([2.0, 3.0, 3.5, 1.0])
    assert last == pytest.approx(11.0)


def test_fcfs_queue_orders_by_arrival():
    lat, last = fcfs_latencies([5.0, 0.0], [1.0, 1.0])
    assert lat == pytest.approx([1.0, 1.0]) and last == pytest.approx(6.0)
