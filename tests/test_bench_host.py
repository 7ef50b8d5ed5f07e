"""Host-side logic of bench.py (no GPU): the one-GPU contract and the number
of evaluations captured per HIP graph."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("steps, requested, expect", [
    (200, 0, 50), (40, 0, 40), (60, 0, 30), (12, 0, 12), (53, 0, 1), (1, 0, 1), (400, 40, 40),
])
def test_graph_holds_a_divisor_of_the_steps(steps, requested, expect):
    G = bench.graph_evals(steps, requested)
    assert G == expect and steps % G == 0


@pytest.mark.parametrize("steps, requested", [(10, 4), (0, 0)])
def test_graph_evals_rejects_a_non_divisor(steps, requested):
    with pytest.raises(SystemExit):
        bench.graph_evals(steps, requested)


def test_algorithmic_bytes_and_flops_per_launch():
    """m in + h out in FP32 plus the unique six-component FP32 tensor on the
    (nx+1)(ny+1) quadrant, once per stack: 69.65 MB for 256^2 x 8, 1.674 GB
    for 64 states of 512^2 x 4, 102.9 MB per 256^2 x 10 candidate."""
    assert bench.algorithmic_bytes(256, 256, 8, 1) == 24 * 256 * 256 * 8 + 24 * 257 * 257 * 36
    assert abs(bench.algorithmic_bytes(256, 256, 8, 1) / 1e6 - 69.65) < 0.01
    assert abs(bench.algorithmic_bytes(512, 512, 4, 64) / 1e9 - 1.674) < 0.001
    assert abs(bench.algorithmic_bytes(256, 256, 10, 16, 16) / 16 / 1e6 - 102.9) < 0.1
    # mixing: 36 nz^2 flops per frequency of the (nx+1) x 2ny half spectrum
    f8 = bench.algorithmic_flops(256, 256, 8, 1)
    f0 = bench.algorithmic_flops(256, 256, 8, 1) - 36 * 64 * 257 * 512
    assert 0.7e9 < f8 < 0.76e9 and f0 > 0


def test_distinct_tensor_bytes():
    """The C5 line beside the per-stack formula: 16 states of 256^2 x 10 and
    the 205 distinct pair tensors of the 16 candidates, 0.577 GB; with one
    stack and all pairs distinct the two counts agree."""
    r = bench.with_distinct_tensor({"kernel_ms": 1.0}, 256, 256, 10, 16, 205)
    assert r["alg_bytes_distinct"] == 16 * 24 * 256 * 256 * 10 + 24 * 257 * 257 * 205
    assert abs(r["alg_bytes_distinct"] / 1e9 - 0.577) < 0.001
    assert abs(r["frac_distinct"] - r["alg_bytes_distinct"] / 1e-3 / 8e12) < 1e-12
    r1 = bench.with_distinct_tensor({"kernel_ms": 1.0}, 256, 256, 8, 1, 36)
    assert r1["alg_bytes_distinct"] == bench.algorithmic_bytes(256, 256, 8, 1)


def test_percentiles():
    p = bench.percentiles(np.arange(1, 101, dtype=float))
    assert p["median"] == 50.5 and p["n"] == 100 and p["p10"] < p["median"] < p["p90"]
