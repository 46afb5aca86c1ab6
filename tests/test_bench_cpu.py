"""The benchmark's host-side contract, without a GPU: it runs on one GPU only and says
so, and the traffic record it reads belongs to the kernel sources it was taken on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_traffic_is_reported_only_for_the_kernel_sources_it_was_taken_on():
    for prec in ("f32", "f64"):
        with open(bench.TRAFFIC_FILES[prec]) as f:
            t = json.load(f)
        assert t["bytes_per_launch"] == t["bytes_read"] + t["bytes_written"]
        # the L2 egress of the force pass is at least its algorithmic bytes
        r = 4 if prec == "f32" else 8
        assert t["bytes_per_launch"] >= bench.BYTES_FACTORED(r) * 32 * 32 * 32 * 64 * 4
        want = t["bytes_per_launch"] if t["source_sha256"] == bench.kernel_source_hash() else None
        assert bench.measured_traffic(prec) == want
