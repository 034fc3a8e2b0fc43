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


def _write_csv(path, header, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        wr = csv.writer(f)
        wr.writerow(header)
        wr.writerows(rows)


def _fake_profile(d, lag, lb_fetch_kib, lb_us, with_copy):
    """rocprofv3-shaped CSVs of one profiled headline run: the level-blocked
    kernel (one launch per run) and p x SpMV (8 launches), plus the bench
    line that names the tuning."""
    lb = "void mpk::lb_sell_kernel<double, 1>(mpk::(anonymous namespace)::LBParams, mpk::Coefs)"
    sp = "void mpk::spmv_sell_kernel<double, 1, false>(mpk::DevMatrix, mpk::PowerIO, int)"
    _write_csv(os.path.join(d, "trace", "run_kernel_stats.csv"),
               ["Name", "Calls", "AverageNs", "TotalDurationNs"],
               [[lb, 3, lb_us * 1e3, 3 * lb_us * 1e3], [sp, 24, 150e3, 24 * 150e3]])
    for sub, counter, lbv, spv in (("fetch", "FETCH_SIZE", lb_fetch_kib, 300000.0),
                                   ("write", "WRITE_SIZE", 16000.0, 16384.0),
                                   ("tcc", "TCC_HIT_sum", 100.0, 300.0)):
        rows = [[lb, i, counter, lbv] for i in range(3)] + [[sp, 10 + i, counter, spv]
                                                             for i in range(24)]
        if sub == "tcc":
            rows += [[lb, i, "TCC_MISS_sum", 900.0] for i in range(3)]
            rows += [[sp, 10 + i, "TCC_MISS_sum", 700.0] for i in range(24)]
        _write_csv(os.path.join(d, sub, "run_counter_collection.csv"),
                   ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"], rows)
    if with_copy:   # a 1 GiB copy reading 2^19 KiB and writing 2^20 KiB as counted
        cp = "__amd_rocclr_copyBuffer"
        _write_csv(os.path.join(d, "cfetch", "copy_counter_collection.csv"),
                   ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
                   [[cp, 1, "FETCH_SIZE", float(1 << 19)]])
        _write_csv(os.path.join(d, "cwrite", "copy_counter_collection.csv"),
                   ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
                   [[cp, 1, "WRITE_SIZE", float(1 << 20)]])
    import json
    line = {"config": {"p": 8, "workload": "test stencil"},
            "roofline": {"run_key": f"level_blocked:wave:16384:64:{lag}:1024:none"},
            "plan": {"launches_per_run": 1}, "baseline_pxspmv": {"reorder": "none"},
            "command": f"python3 bench.py --lag {lag}"}
    with open(os.path.join(d, "trace.log"), "w") as f:
        f.write("[bench] log line\n" + json.dumps(line) + "\n")


def test_counter_reduction_merges_tunings(tmp_path):
    a, b = str(tmp_path / "prof"), str(tmp_path / "prof2")
    _fake_profile(a, 128, 2000000.0, 980.0, True)
    _fake_profile(b, 192, 2100000.0, 990.0, False)
    red = bench.reduce_counter_dirs([a, b])
    assert red["fetch_scale"] == 2.0 and red["write_scale"] == 1.0
    runs = red["runs"]
    assert set(runs) == {"level_blocked:wave:16384:64:128:1024:none",
                         "level_blocked:wave:16384:64:192:1024:none", "pxspmv:none"}
    r128 = runs["level_blocked:wave:16384:64:128:1024:none"]
    assert r128["l2_egress_bytes_per_run"] == int((2000000.0 * 2 + 16000.0) * 1024)
    assert r128["avg_launch_us"] == 980.0 and r128["l2_hit_rate"] == 0.1
    r192 = runs["level_blocked:wave:16384:64:192:1024:none"]
    assert r192["l2_egress_bytes_per_run"] == int((2100000.0 * 2 + 16000.0) * 1024)
    sp = runs["pxspmv:none"]
    assert sp["launches_per_run"] == 8
    assert sp["l2_egress_bytes_per_run"] == 8 * int((300000.0 * 2 + 16384.0) * 1024)
    assert red["commands"] == ["python3 bench.py --lag 128", "python3 bench.py --lag 192"]
    md = bench.counters_markdown([a, b], red)
    assert "--lag 128" in md and "--lag 192" in md and f"-d {b}/fetch" in md
    assert "level_blocked:wave:16384:64:192:1024:none" in md
