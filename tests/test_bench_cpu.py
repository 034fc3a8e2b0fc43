"""The bench script's contract on the CPU: more than one GPU is refused with a
message, and the algorithmic byte counts follow their definitions."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    n, nnz, p, R = 10, 30, 4, 2
    A = 4 * (n + 1) + 12 * nnz
    V = 8 * n * R
    assert bench.algorithmic_bytes(n, nnz, p, R, 8, "trad") == p * (A + 2 * V)
    assert bench.algorithmic_bytes(n, nnz, p, R, 8, "lb") == A + V + p * V
    assert bench.algorithmic_bytes(n, nnz, p, R, 4, "lb") == 4 * (n + 1) + 8 * nnz + V + p * V
    assert bench.algorithmic_bytes(n, nnz, p, R, 8, "trad", n) == p * (A + 2 * V + 4 * n)
