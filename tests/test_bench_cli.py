"""Host-side checks of bench.py: the one-GPU contract and the algorithmic flop
counts its rooflines divide by (no GPU needed)."""
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
    assert "one GPU" in r.stderr and r.stdout == ""


def test_flops_per_evaluation():
    # identity patch: per tap 3 flops per channel (difference, multiply-add)
    # plus one weight multiply per gradient channel; distorted patch: each
    # channel value bilinear first (three lerps of a subtract and an FMA)
    assert bench.flops_per_eval("identity", 4, 5) == 81 * (3 * 5 + 2) == 1377
    assert bench.flops_per_eval("distorted", 4, 5) == 81 * (12 * 5 + 2) == 5022
    assert bench.flops_per_eval("identity", 3, 3) == 49 * 9
    assert bench.flops_per_eval("distorted", 1, 3) == 9 * 36
