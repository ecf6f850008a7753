"""The benchmark's algorithmic byte/flop model, roofline arithmetic and
contract checks that need no GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_history_bytes_of_the_torus():
    """Four folded lags of three 3072 x 3072 FP64 blocks, plus the ring and the
    RHS slice read and the result written: the bytes per history launch."""
    import bench
    nbytes, flops = bench.history_model(3072, 6144, 5, 1, 0, 2)
    assert nbytes == 4 * 3 * 3072 * 3072 * 8 + 8 * (4 * 6144 + 2 * 6144) == 906264576
    assert flops == 2 * 4 * 3072 * 3072 * 4
    # mixed: FP32 lags plus the FP32 low parts of two lags
    mb, mf = bench.history_model(1920, 3840, 21, 16, 1, 2)
    assert mb == 3 * 1920 * 1920 * (20 + 2) * 4 + 8 * (20 * 3840 * 16 + 2 * 3840 * 16)
    assert mf == 2 * 4 * 1920 * 1920 * 16 * 20


def test_roofline_arithmetic():
    import bench
    r = bench.roofline("k", 8e9, 0.0, 1e6, "f64", False, None)      # 8 GB in 1 s
    assert r["bound"] == "hbm" and r["achieved"] == 8.0 and r["frac"] == 0.001
    r = bench.roofline("k", 1.0, 78.6e12, 1e6, "f64", True, None)   # 78.6 TFLOP in 1 s
    assert r["bound"] == "mfma" and r["achieved"] == 78.6 and r["frac"] == 1.0


def test_committed_traffic_agrees_with_the_model():
    """profiles/traffic.json: HBM bytes per dispatch from the counter runs,
    used by the bench only while the kernel's source is unchanged; where it is
    used, it is within 10% of the algorithmic bytes."""
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    assert t["kernels"]
    model = bench.history_model(3072, 6144, 5, 1, 0, 2)[0]
    got = bench.measured_traffic("k_history_rows<4>", "torus_3072")
    if got is not None:
        assert abs(got / model - 1) < 0.1


def test_several_gpus_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout == ""
