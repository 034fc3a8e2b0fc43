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


def test_flush_bytes_follow_the_flush_plan():
    # a sum's first flush writes it (V), every later one reads and writes it
    assert bench.flush_bytes([0.0, 0.0, 0.0], 1) == 1          # all zero: written once
    assert bench.flush_bytes([1.0, 0.0, 0.0], 1) == 1          # one flush
    # Chebyshev real part for M = 16: terms 0, 2, ..., 16 flushed at 2, 6, 10, 14, 16
    wa = [1.0 if k % 2 == 0 else 0.0 for k in range(17)]
    assert bench.flush_bytes(wa, 1) == 1 + 2 * 4
    # imaginary part: terms 1, 3, ..., 15 flushed at 3, 7, 11, 15
    wb = [1.0 if k % 2 else 0.0 for k in range(17)]
    assert bench.flush_bytes(wb, 1) == 1 + 2 * 3
    # every weight nonzero: flushes at 2, 5, 8, ... (terms k..k+2 together)
    assert bench.flush_bytes([1.0] * 9, 1) == 1 + 2 * 2        # p = 8: 2, 5, 8
