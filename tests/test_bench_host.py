"""Host-side logic of bench.py (no GPU): the one-GPU contract and the number
of evaluations captured per HIP graph."""
import os
import subprocess
import sys

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
    (200, 0, 10), (40, 0, 10), (12, 0, 6), (7, 0, 7), (13, 0, 1), (1, 0, 1), (400, 40, 40),
])
def test_graph_holds_a_divisor_of_the_steps(steps, requested, expect):
    G = bench.graph_evals(steps, requested)
    assert G == expect and steps % G == 0


@pytest.mark.parametrize("steps, requested", [(10, 4), (0, 0)])
def test_graph_evals_rejects_a_non_divisor(steps, requested):
    with pytest.raises(SystemExit):
        bench.graph_evals(steps, requested)
