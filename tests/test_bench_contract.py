"""Host-side parts of the benchmark's contract (no GPU): one GPU only, and
the counter-based traffic field is reported only for the kernel sources the
counters were taken on."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
import rodsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert r.stdout == ""
    assert "one GPU" in r.stderr


def test_traffic_is_null_for_other_kernel_sources(tmp_path):
    t = {"source_hash": bench.source_hash(),
         "kernels": {"rod": {"name": "k_rod<2,true>", "hbm_bytes_per_launch": 123456}}}
    good = tmp_path / "good.json"
    good.write_text(json.dumps(t))
    assert bench.measured_traffic("rod", str(good)) == 123456
    t["source_hash"] = "0" * 16
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps(t))
    assert bench.measured_traffic("rod", str(stale)) is None
    assert bench.measured_traffic("rod", str(tmp_path / "missing.json")) is None


def test_crosslinkers_in_a_ball_are_inside_and_seeded():
    c = (5.0, 5.0, 5.0)
    a = rodsynth.crosslinker_positions_ball(5000, c, 2.0, seed=3)
    b = rodsynth.crosslinker_positions_ball(5000, c, 2.0, seed=3)
    assert np.array_equal(a, b)
    r = np.linalg.norm(a - np.asarray(c), axis=1)
    assert r.max() <= 2.0
    # uniform in the ball: P(r < R/2) = 1/8
    assert abs(np.mean(r < 1.0) - 0.125) < 0.02
