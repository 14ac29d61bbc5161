"""Host-side pieces of bench.py: the output contract, the roofline arithmetic
and the refusal of multi-GPU runs (no GPU needed)."""
import json
import math
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_finite_json_makes_strict_json():
    out = bench.finite_json({"a": float("nan"), "b": [1.5, float("-inf")], "c": {"d": (2.0, math.inf)},
                             "e": "x", "f": 3})
    s = json.dumps(out, allow_nan=False)
    assert json.loads(s) == {"a": None, "b": [1.5, None], "c": {"d": [2.0, None]}, "e": "x", "f": 3}


def test_roofline_from_trace_arithmetic():
    # two kernels; the one with the larger total time is dominant
    recs = ([{"kernel": "gemm_f64_128x128", "ms": 2.0, "flops": 1.0e11, "bytes": 3.0e8}] * 4
            + [{"kernel": "leaf_gj_panel", "ms": 0.1, "flops": 1.0e6, "bytes": 0.0}] * 8)
    roof, breakdown = bench.roofline_from_trace(recs, n_steps=2)
    assert roof["kernel"] == "gemm_f64_128x128"
    assert roof["launches"] == 4
    assert abs(roof["avg_launch_ms"] - 2.0) < 1e-12
    assert abs(roof["achieved"] - 50.0) < 1e-9          # 1e11 flop / 2 ms = 50 TFLOP/s
    assert roof["peak"] == bench.PEAK_FP64_TFLOPS
    assert abs(roof["frac"] - round(50.0 / 78.6, 4)) < 1e-12
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s"
    assert breakdown["gemm_f64_128x128"]["launches_per_step"] == 2
    assert abs(breakdown["leaf_gj_panel"]["ms_per_step"] - 0.4) < 1e-9


def test_measured_traffic_is_keyed_to_the_source():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["gemm_f64_128x128"]
    assert rec["source"] == "paper_1801_04723_amd/csrc/gemm.hip"
    assert rec["bytes_per_launch"] > 0
    # an unknown kernel has no measured traffic
    assert bench.measured_traffic("no_such_kernel") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
