"""Benchmark: level-blocked matrix power kernel vs p x SpMV on one MI355X.

Workload: 3D 27-point stencil on a 128^3 grid (n = 2,097,152, nnz =
55,742,968, truncated boundary, diagonal 26 and off-diagonals -1, FP64
values), x uniform in [-1, 1) from seed 1002, p = 8 powers, one right-hand
side.  One step = one call that produces all p powers, inputs already
resident in HBM.  Prints ONE JSON line on stdout (progress goes to stderr).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-serve]

The level-blocked run uses the plan's autotuned schedule (BFS and original
order are both tried; the faster is reported).  A serving session on the
six-matrix pool (2D/3D stencils and Anderson lattices, N from 1e4 to 4.1e6)
measures the saturated request rate, then replays 512 Poisson arrivals at a
fixed rate (--serve-rate) and reports p50/p99 latency overall and per matrix.
With the CPU leg on, each power of the headline result is compared with the
FP64 oracle.

The roofline object describes the level-blocked run: algorithmic bytes
(matrix once, x once, p output vectors; see algorithmic_bytes) divided by
the mean duration of one run, measured with HIP events recorded on the
stream the kernels are launched on.  Measured traffic (bytes at L2 egress,
which include Infinity Cache hits) is taken from the committed counter
summary when it was recorded for the current kernel source (same SHA-256)
and the same tuning, else reported as null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

_ROOT = os.path.dirname(os.path.abspath(__file__))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

METRIC = "MPK Gflop/s & HBM bytes vs p×SpMV at p=8 (1 GPU); serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "stencil3d27_128_p8"
WORKLOAD_TEXT = {
    "stencil3d27_128_p8": ("3D 27-point stencil 128^3 (truncated), {vb} CSR, x U[-1,1) seed 1002, "
                           "p=8, 1 RHS, level-blocked MPK, caller's order", 64),
    "banded_4m_p6": ("banded random N=2^22 (half-width 5000, ~16 nnz/row, 64k-window "
                     "permutation), {vb} CSR, x U[-1,1) seed 1003, p=6, 1 RHS", 64),
    "anderson160_cheb16_r8": ("Anderson 160^3 periodic (W=16.5, /14.25), {vb} CSR, Chebyshev "
                              "recurrence p=16, 8 random-sign RHS seed 1004", 32),
    "stencil3d27_64_p16_r16": ("3D 27-point stencil 64^3 (truncated), {vb} CSR, x U[-1,1) seed "
                               "1006, p=16, 16 RHS", 64),
}
KERNEL_SRC = os.path.join(_ROOT, "paper_2405_12525_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(_ROOT, "profiles", "traffic_{workload}_fp{vb}.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(n, nnz, p, R, value_bytes, kind, perm_rows=0):
    """Bytes a run must move at minimum (4-byte indices, no write-allocate).

    A = 4(n+1) + (4 + value_bytes) nnz is the CSR, V = 8 n R one vector block.
    p x SpMV streams A and reads / writes one block per power: p (A + 2V).
    Level-blocked: A once, x once, p output blocks: A + V + p V.  perm_rows
    adds 4 bytes per row and pass for the output-row permutation when results
    are written in the caller's order.
    """
    A = 4 * (n + 1) + (4 + value_bytes) * nnz
    V = 8 * n * R
    if kind == "trad":
        return p * (A + 2 * V + perm_rows * 4)
    return A + V + p * V + perm_rows * 4


def per_power_rel_err(got, ref):
    """Relative error of each power against the FP64 oracle: for power k the
    largest, over right-hand sides, of ||got_k - ref_k||_2 / ||ref_k||_2."""
    import numpy as np
    p, R = ref.shape[0], ref.shape[-1]
    num = np.linalg.norm((got - ref).reshape(p, -1, R), axis=1)
    den = np.linalg.norm(ref.reshape(p, -1, R), axis=1)
    return [float(v) for v in np.max(num / np.where(den > 0, den, 1.0), axis=1)]


def time_calls(fn, steps, warmup, torch, stream):
    """Per-call durations from events recorded on `stream` (the launch stream)."""
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            fn()
        stream.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            starts[i].record(stream)
            fn()
            ends[i].record(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return dict(median_ms=statistics.median(ms), mean_ms=statistics.fmean(ms), min_ms=min(ms),
                total_ms=sum(ms), wall_s=wall)


def measured_traffic(workload, vb, run_key):
    """Bytes per run at L2 egress from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the same counters
    read for a 1 GiB copy), if it was taken for the current kernel source and
    this tuning; else None."""
    try:
        with open(TRAFFIC_FILE.format(workload=workload, vb=vb)) as f:
            t = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    run = t.get("runs", {}).get(run_key)
    if t.get("kernels_sha256") != sha or not run:
        return None
    return run.get("l2_egress_bytes_per_run")


SERVE_HW_QUEUES = 16   # hardware queues for the serving session (one per stream, with room)


def serving(torch, mpk, w, rates, n_requests=512):
    """The saturated rate first (all requests at t = 0), then Poisson arrivals
    at each fixed rate in `rates` (the first is reported at the top level).
    Each pool plan is autotuned once (p = 16, 4 RHS) with tasks from the
    shared counter (the order the server runs them in) and serves through the
    level-blocked kernels only where they were at least 5% faster than the
    p x SpMV kernels at that shape: a persistent launch holds its workgroups
    for the whole run, while p x SpMV's launches free the compute units for
    other batches between powers (the results are the same bit for bit); one
    stream per matrix."""
    from paper_2405_12525_amd import serve
    t0 = time.perf_counter()
    specs = w.serving_pool_specs()
    mats = [w.build_pool_matrix(s) for s in specs]
    plans = [mpk.Plan(A) for A in mats]
    use_base = []
    stream = torch.cuda.Stream()
    for P in plans:
        xt = torch.rand((P.n, 4), device="cuda", dtype=torch.float64)
        Yt = torch.empty((16, P.n, 4), device="cuda", dtype=torch.float64)
        P.tune(dynamic_tickets=1)
        lb_ms = P.autotune(xt, 16, Yt, reps=3, stream=stream)["ms"]
        tr_ms = time_calls(lambda: P.run_baseline(xt, 16, Yt, stream=stream), 3, 1, torch,
                           stream)["mean_ms"]
        use_base.append(lb_ms > 0.95 * tr_ms)
        del xt, Yt
    log(f"[bench] serving pool ready in {time.perf_counter() - t0:.1f}s: "
        + ", ".join(f"{k}{sz} n={A.n}" for (k, sz), A in zip(specs, mats)))
    names = [f"{k}{sz}" for k, sz in specs]

    def requests(rate):
        reqs = []
        for s in w.serving_requests(n_requests, rate_per_s=rate, seed=5005, pool_size=len(plans)):
            g = torch.Generator(device="cuda")
            g.manual_seed(s["x_seed"])
            n = plans[s["matrix"]].n
            x = torch.rand((n, s["R"]), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
            reqs.append(serve.Request(id=s["id"], arrival=s["t"], matrix=s["matrix"], p=s["p"], x=x))
        return reqs

    def paced(st, rate):
        return {"rate_rps": round(rate, 1), "p50_ms": round(st["p50_ms"], 3),
                "p99_ms": round(st["p99_ms"], 3),
                "queue_p50_ms": round(st["queue_p50_ms"], 3),
                "queue_p99_ms": round(st["queue_p99_ms"], 3),
                "device_p50_ms": round(st["device_p50_ms"], 3),
                "device_p99_ms": round(st["device_p99_ms"], 3),
                "throughput_rps": round(st["throughput_rps"], 1),
                "gflops": round(st["gflops"], 1), "mean_batch": round(st["mean_batch"], 2),
                "by_matrix": {names[m]: {k: (round(x, 3) if isinstance(x, float) else x)
                                         for k, x in v.items()}
                              for m, v in st["by_matrix"].items()}}

    # one stream per matrix (at most one batch of a matrix in flight); a
    # fixed stream per matrix by size (Server.size_lanes) was measured no
    # better: its shared stream made the small matrices wait longer
    srv = serve.Server(plans, n_streams=len(plans), use_baseline=use_base)
    srv.prepare(32)
    warm = requests(1000.0)[:24]
    srv.serve(warm, realtime=False, keep=False)
    reqs = requests(1000.0)
    sat = serve.summarize(srv.serve(reqs, realtime=False, keep=False), reqs, plans)
    del reqs
    runs = []
    for rate in rates:
        reqs = requests(rate)
        res = srv.serve(reqs, realtime=True, keep=False)
        st = serve.summarize(res, reqs, plans)
        del res, reqs
        log(f"[bench] serving at {rate:.0f} req/s: p50 {st['p50_ms']:.2f} ms p99 "
            f"{st['p99_ms']:.2f} ms, mean batch {st['mean_batch']:.2f}")
        runs.append(paced(st, rate))
    for P in plans:
        P.close()
    log(f"[bench] serving: saturated {sat['throughput_rps']:.0f} req/s")
    out = {"requests": n_requests, "rate_rule": "fixed (--serve-rate)", **runs[0],
           "kernels": {names[m]: "p x SpMV" if b else "level-blocked"
                       for m, b in enumerate(use_base)},
           "streams": len(plans),
           "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES") or 4),
           "max_inflight_per_matrix": 1,
           "saturated_rps": round(sat["throughput_rps"], 1),
           "saturated_gflops": round(sat["gflops"], 1),
           "saturated_mean_batch": round(sat["mean_batch"], 2)}
    if len(runs) > 1:
        out["other_rates"] = runs[1:]
    return out


def other_configs(torch, mpk, w, steps, warmup, stream, with_oracle):
    """The banded random matrix (FP64 and FP32 values, p = 6), the Anderson
    lattice (Chebyshev p = 16, 8 RHS, FP32 values) and a 64^3 27-point
    stencil with 16 RHS (p = 16): autotuned level-blocked run vs p x SpMV in
    the faster order.  With the CPU leg on (with_oracle), also each power's
    relative error against the FP64 oracle (the larger of the two orders)."""
    out = {}
    if with_oracle:
        import oracle
    for name, vbs in (("banded_4m_p6", (64, 32)), ("anderson160_cheb16_r8", (32,)),
                      ("stencil3d27_64_p16_r16", (64,))):
        A, x, p, kind = w.config(name)
        R = x.shape[1]
        xd = torch.from_numpy(x).cuda()
        cheb = kind == "chebyshev"
        coefs = mpk.chebyshev_coefficients(p) if cheb else None
        ref = None
        if with_oracle:
            ref = oracle.recur(A, x, *coefs) if cheb else oracle.powers(A, x, p)
        flop = mpk.flops(A.nnz, A.n, p, R, recur=cheb)
        extra_v = p - 1 if cheb else 0   # y_{k-1} read again by the recurrence (powers 2..p)
        Y = torch.empty((p, A.n, R), dtype=torch.float64, device="cuda")
        for vb in vbs:
            best = {}
            for ro in ("bfs", "none"):
                P = mpk.Plan(A, reorder=ro, value_bits=vb)
                if cheb:
                    lbf = lambda: P.run_recur(xd, *coefs, Y=Y, stream=stream)
                    trf = lambda: P.run_baseline_recur(xd, *coefs, Y=Y, stream=stream)
                else:
                    lbf = lambda: P.run(xd, p, Y, stream=stream)
                    trf = lambda: P.run_baseline(xd, p, Y, stream=stream)
                tr = time_calls(trf, steps, warmup, torch, stream)["median_ms"]
                tq = P.autotune(xd, p, Y, reps=3, recur=cheb, stream=stream)
                lb = time_calls(lbf, steps, warmup, torch, stream)["median_ms"]
                P.sync()
                if ref is not None:
                    rel = per_power_rel_err(Y.cpu().numpy(), ref)
                    best["rel"] = [max(a, b) for a, b in zip(best.get("rel", rel), rel)]
                tuning = {k: tq[k] for k in ("schedule", "chunk_nnz", "lag", "workgroups",
                                             "seg_powers", "skip_ahead", "dynamic_tickets")}
                for key, ms in (("trad", tr), ("lb", lb)):
                    if key not in best or ms < best[key][0]:
                        best[key] = (ms, ro, tq["schedule"] if key == "lb" else None, tuning)
                P.close()
            tag = f"{name}_fp{vb}"
            vbytes = 8 * A.n * R
            trad_b = algorithmic_bytes(A.n, A.nnz, p, R, vb // 8, "trad") + extra_v * vbytes
            lb_b = algorithmic_bytes(A.n, A.nnz, p, R, vb // 8, "lb")
            out[tag] = {"n": A.n, "nnz": A.nnz, "p": p, "nrhs": R, "kind": kind,
                        "lb_ms": round(best["lb"][0], 4), "lb_reorder": best["lb"][1],
                        "lb_schedule": best["lb"][2], "lb_tuning": best["lb"][3],
                        "lb_gflops": round(flop / best["lb"][0] / 1e6, 1),
                        "pxspmv_ms": round(best["trad"][0], 4), "pxspmv_reorder": best["trad"][1],
                        "pxspmv_gflops": round(flop / best["trad"][0] / 1e6, 1),
                        "speedup_vs_pxspmv": round(best["trad"][0] / best["lb"][0], 3),
                        "rel_err_per_power_vs_fp64_oracle": best.get("rel"),
                        "pxspmv_roofline": {"bound": "hbm", "algorithmic_bytes": trad_b,
                                            "achieved_GBs": round(trad_b / best["trad"][0] / 1e6, 1),
                                            "frac": round(trad_b / best["trad"][0] / 1e6 / HBM_PEAK_GBS, 4)},
                        "lb_roofline": {"bound": "hbm", "algorithmic_bytes": lb_b,
                                        "achieved_GBs": round(lb_b / best["lb"][0] / 1e6, 1),
                                        "frac": round(lb_b / best["lb"][0] / 1e6 / HBM_PEAK_GBS, 4)},
                        "tolerance": 1e-12 if vb == 64 else 1e-5}
            rel = max(best["rel"]) if "rel" in best else float("nan")
            log(f"[bench] {tag}: level-blocked {best['lb'][0]:.3f} ms ({best['lb'][2]}, "
                f"{best['lb'][1]}), p x SpMV {best['trad'][0]:.3f} ms, max rel err {rel:.2e}")
        del Y, xd
    return out


def flush_bytes(wts, V):
    """HBM bytes of one weighted sum: the kernels flush its pending nonzero
    terms k..min(k+2, p) at power min(k+2, p), the first flush writing the
    sum (V) and each later one reading and writing it (2 V)."""
    p = len(wts) - 1
    k, n_flush = 0, 0
    while True:
        while k <= p and wts[k] == 0.0:
            k += 1
        if k > p:
            break
        n_flush += 1
        k = min(k + 2, p) + 1
    return V if n_flush == 0 else V + 2 * V * (n_flush - 1)


def time_step(torch, mpk, w, steps, warmup, stream, with_oracle=True, tuning=None):
    """One Chebyshev time step exp(-i dt H) psi on the Anderson lattice (160^3,
    FP32 values, 4 complex states as 8 real columns, M = 16, dt = 1): the
    weighted sums accumulated in the kernels over a two-vector ring, level-
    blocked and as p x SpMV, against the recurrence that writes all M vectors
    (without even summing them).  The result is checked bit for bit against
    the oracle's sums with the same weights when the CPU leg is on
    (with_oracle).  tuning: a fixed level-blocked tuning instead of the
    autotuner's (profiling)."""
    import numpy as np
    A, x, _, _ = w.config("anderson160_cheb16_r8")
    M, dt = 16, 1.0
    n, R = A.n, x.shape[1]
    xd = torch.from_numpy(x).cuda()
    al, be, ga, wa, wb = mpk.cheb_time_coefficients(M, dt)
    # the lattice's own order: faster than BFS order for both forms here
    P = mpk.Plan(A, value_bits=32, reorder="none")
    Y = torch.empty((M, n, R), dtype=torch.float64, device="cuda")
    if tuning is None:
        tq = P.autotune(xd, M, Y, reps=3, recur=2, stream=stream)   # the weighted-sum kernels
    else:
        tq = P.tune(**tuning)
    out = torch.empty_like(xd)
    acc = torch.empty((2, n, R), dtype=torch.float64, device="cuda")
    work = torch.empty((2, n, R), dtype=torch.float64, device="cuda")

    def fused(baseline):
        run = P.run_baseline_poly if baseline else P.run_poly
        run(xd, wa, wb, al, be, ga, acc=acc, work=work, stream=stream)
        P.combine_complex(acc, out, stream=stream)
    lb = time_calls(lambda: fused(False), steps, warmup, torch, stream)["median_ms"]
    P.sync()
    got_lb = out.cpu().numpy()
    tr = time_calls(lambda: fused(True), steps, warmup, torch, stream)["median_ms"]
    P.sync()
    got_tr = out.cpu().numpy()
    graphs = {}
    for name, base in (("level_blocked", False), ("pxspmv", True)):
        gout = torch.empty_like(xd)
        G = P.capture_time_step(xd, dt, M, gout, baseline=base)
        graphs[name] = round(time_calls(lambda: G.launch(stream=stream), steps, warmup, torch,
                                        stream)["median_ms"], 4)
        stream.synchronize()
        graphs[name + "_equal"] = bool(np.array_equal(gout.cpu().numpy(), got_lb))
        G.close()
    full = time_calls(lambda: P.run_recur(xd, al, be, ga, Y=Y, stream=stream), steps, warmup,
                      torch, stream)["median_ms"]
    full_tr = time_calls(lambda: P.run_baseline_recur(xd, al, be, ga, Y=Y, stream=stream), steps,
                         warmup, torch, stream)["median_ms"]
    P.sync()
    exact = None
    if with_oracle:
        import oracle
        ra, rb = oracle.poly_sums(A, x, al, be, ga, wa, wb, value_bits=32)
        ref = oracle.combine_complex(ra, rb)
        exact = bool(np.array_equal(got_lb, ref) and np.array_equal(got_tr, ref))
    def norms(v):  # per complex state, with an exactly rounded sum of squares
        import math
        sq = v[:, 0::2] ** 2 + v[:, 1::2] ** 2
        return np.array([math.sqrt(math.fsum(sq[:, j])) for j in range(sq.shape[1])])
    norm_drift = float(np.max(np.abs(norms(got_lb) / norms(x) - 1.0)))
    P.close()
    del Y, acc, work, out, xd
    V = 8 * n * R
    Ab = 4 * (n + 1) + 8 * A.nnz
    flop = mpk.flops(A.nnz, n, M, R, recur=True) + 2.0 * n * R * (M + 1) + n * R
    # p x SpMV: A, the gathered y_{k-1} and the written y_k per power, y_{k-2}
    # read from the second power on, the sums' flushes (a sum's first flush
    # writes it, every later one reads and writes it), then the combination
    # (2 V read, V written)
    trad_b = M * Ab + M * V + (M - 1) * V + M * V + flush_bytes(wa, V) + flush_bytes(wb, V) \
        + 3 * V
    # level-blocked ideal: A, x, the two ring slots and the two sums once
    lb_b = Ab + V + 2 * V + 2 * V + 3 * V
    res = {"n": n, "nnz": A.nnz, "M": M, "dt": dt, "states": R // 2, "real_columns": R,
           "values": "fp32", "schedule": tq["schedule"], "gflops_flop_count": flop,
           "tuning": {k: tq[k] for k in ("schedule", "chunk_nnz", "lag", "workgroups",
                                         "seg_powers", "dynamic_tickets")},
           "lb_fused_ms": round(lb, 4), "lb_fused_gflops": round(flop / lb / 1e6, 1),
           "pxspmv_fused_ms": round(tr, 4), "pxspmv_fused_gflops": round(flop / tr / 1e6, 1),
           "hip_graph_ms": graphs,
           "recurrence_writing_all_M_vectors_ms": {"level_blocked": round(full, 4),
                                                   "pxspmv": round(full_tr, 4)},
           "reorder": "none",
           "device_vectors_fused": 4, "device_vectors_unfused": M,
           "bit_identical_to_oracle_sums": exact, "norm_drift": norm_drift,
           "pxspmv_roofline": {"bound": "hbm", "algorithmic_bytes": trad_b,
                               "achieved_GBs": round(trad_b / tr / 1e6, 1),
                               "frac": round(trad_b / tr / 1e6 / HBM_PEAK_GBS, 4)},
           "lb_roofline": {"bound": "hbm", "algorithmic_bytes": lb_b,
                           "achieved_GBs": round(lb_b / lb / 1e6, 1),
                           "frac": round(lb_b / lb / 1e6 / HBM_PEAK_GBS, 4)}}
    log(f"[bench] time step: level-blocked fused {lb:.3f} ms ({tq['schedule']}), "
        f"p x SpMV fused {tr:.3f} ms, graphs {graphs}, "
        f"recurrence writing all vectors {full:.3f} / {full_tr:.3f} ms, "
        f"exact {exact}")
    return res


def cpu_baseline(A, x, p, budget_s=20.0):
    """The CPU oracle on all host cores: whole runs of the workload, bounded in
    time; also one core, for reference (3 runs).  Returns the summary and the
    oracle's powers (p, n, R) of the last run."""
    import oracle
    nthreads = oracle.threads()
    t1 = []
    for _ in range(3):   # first: the thread count set here holds until the next call sets it
        t0 = time.perf_counter()
        oracle.powers(A, x, p, nthreads=1)
        t1.append(time.perf_counter() - t0)
    gflops1 = 2.0 * A.nnz * x.shape[1] * p / statistics.median(t1) / 1e9
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        ref = oracle.powers(A, x, p, nthreads=nthreads)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 5:
            break
    med = statistics.median(times)
    gflops = 2.0 * A.nnz * x.shape[1] * p / med / 1e9
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(gflops, 3), "unit": "Gflop/s", "cores": nthreads, "kind": "oracle",
            "sample": f"the full workload (all {p} powers), median of {len(times)} runs "
                      f"({med * 1e3:.0f} ms each), OpenMP over rows on {nthreads} threads of {cpu}",
            "single_thread_value": round(gflops1, 3)}, ref


def bandwidth_sweep(torch, mpk, stream, reps=5):
    """Load-only bandwidth against the working-set size (1 MiB .. 4 GiB), the
    MI355X counterpart of the paper's load-bandwidth curves: 'global' lets
    every workgroup stride over the whole buffer (each XCD's L2 sees all of
    it); 'xcd_local' gives each XCD its own eighth (its L2 sees 1/8).  Each
    point reads at least ~4 GB in one launch; median of `reps` launches timed
    with events on the launch stream."""
    wg = 4096
    buf = torch.ones(1 << 29, dtype=torch.float64, device="cuda")   # 4 GiB
    sink = torch.empty(wg, dtype=torch.float64, device="cuda")
    xcc = torch.empty(wg, dtype=torch.int32, device="cuda")
    rows = []
    for lg in range(20, 33):
        nbytes = 1 << lg
        view = buf[: nbytes // 8]
        passes = max(1, (4 << 30) // nbytes)
        for mode in ("global", "xcd_local"):
            if mode == "global":
                fn = lambda: mpk.probe_load(view, passes=passes, workgroups=wg, sink=sink,
                                            stream=stream)
            else:
                fn = lambda: mpk.probe_load_xcd(view, regions=8, passes=passes, workgroups=wg,
                                                sink=sink, xcc=xcc, stream=stream)
            t = time_calls(fn, reps, 1, torch, stream)
            gbs = nbytes * passes / (t["median_ms"] * 1e-3) / 1e9
            rows.append({"bytes": nbytes, "mode": mode, "passes": passes,
                         "ms": round(t["median_ms"], 4), "GBs": round(gbs, 1)})
            log(f"[bench] probe {mode:9s} {nbytes / 2**20:8.0f} MiB x{passes}: {gbs:8.0f} GB/s")
    ids = xcc.cpu().numpy()
    import numpy as np
    placement = bool(np.array_equal(ids, np.arange(wg) % 8))
    del buf
    return {"workgroups": wg, "threads_per_workgroup": 256, "load_bytes": 16,
            "round_robin_placement": placement, "xcc_ids_seen": sorted(set(int(v) for v in ids)),
            "points": rows}


def _kernel_key(name):
    """Readable kernel name of a rocprofv3 record (no namespaces or argument list)."""
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0].strip()


def reduce_counter_dirs(dirs):
    """reduce_counters of the first directory, with the per-run traffic of
    the others (the same workload profiled at other tunings, without their
    own copy calibration) added to its runs."""
    red = reduce_counters(dirs[0])
    red["dirs"] = [dirs[0]]
    red["commands"] = [red.get("command")]
    for d in dirs[1:]:
        e = reduce_counters(d, (red["fetch_scale"], red["write_scale"]))
        red.setdefault("runs", {}).update(e.get("runs", {}))
        red["dirs"].append(d)
        red["commands"].append(e.get("command"))
    return red


def reduce_counters(d, scales=None):
    """Reduce the rocprofv3 output of one profiled bench configuration:
    d/trace (--kernel-trace --stats), d/fetch (--pmc FETCH_SIZE), d/write
    (--pmc WRITE_SIZE), d/tcc (--pmc TCC_HIT_sum TCC_MISS_sum) and the
    copy-calibration runs d/cfetch, d/cwrite (a 1 GiB device copy, so that
    the counters convert to bytes).  Per kernel: launches, mean duration,
    FETCH/WRITE KiB per launch, the bytes they stand for at L2 egress (reads
    into the L2 from the Infinity Cache or HBM, and writes out of it) and
    the L2 hit rate.  scales: (FETCH_SIZE, WRITE_SIZE) factors taken from
    another directory's calibration instead."""
    import csv
    import glob
    from collections import defaultdict

    def rows(sub, pattern):
        out = []
        for f in sorted(glob.glob(os.path.join(d, sub, "**", pattern), recursive=True)):
            with open(f, newline="") as fh:
                out += list(csv.DictReader(fh))
        return out

    def per_launch(sub):
        acc = defaultdict(lambda: defaultdict(float))
        for r in rows(sub, "*counter_collection.csv"):
            acc[_kernel_key(r["Kernel_Name"])][(r["Dispatch_Id"], r["Counter_Name"])] += \
                float(r["Counter_Value"])
        res = {}
        for k, v in acc.items():
            per = defaultdict(list)
            for (_, cname), val in v.items():
                per[cname].append(val)
            res[k] = {c: sum(x) / len(x) for c, x in per.items()}
        return res

    gib_kib = float(1 << 20)
    cf = per_launch("cfetch").get("__amd_rocclr_copyBuffer", {}).get("FETCH_SIZE")
    cw = per_launch("cwrite").get("__amd_rocclr_copyBuffer", {}).get("WRITE_SIZE")
    fetch_scale = round(gib_kib / cf, 4) if cf else None
    write_scale = round(gib_kib / cw, 4) if cw else None
    if scales is not None:
        fetch_scale, write_scale = scales
    stats = {}
    for r in rows("trace", "*kernel_stats.csv"):
        stats[_kernel_key(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3)
    fetch, write, tcc = per_launch("fetch"), per_launch("write"), per_launch("tcc")
    kernels = {}
    for k in set(fetch) | set(write) | set(tcc):
        if not k.startswith("mpk::") or k not in stats:
            continue
        e = {"launches": stats[k][0], "avg_us": round(stats[k][1], 2)}
        if k in fetch and k in write and fetch_scale and write_scale:
            fk, wk = fetch[k]["FETCH_SIZE"], write[k]["WRITE_SIZE"]
            e.update(fetch_kib_per_launch=round(fk, 1), write_kib_per_launch=round(wk, 1),
                     l2_egress_bytes_per_launch=int((fk * fetch_scale + wk * write_scale) * 1024))
        if k in tcc:
            h, m = tcc[k].get("TCC_HIT_sum", 0.0), tcc[k].get("TCC_MISS_sum", 0.0)
            e.update(tcc_hits_per_launch=int(h), tcc_misses_per_launch=int(m),
                     l2_hit_rate=round(h / (h + m), 4) if h + m else None)
        kernels[k] = e
    out = {"fetch_scale": fetch_scale, "write_scale": write_scale,
           "calibration": "a 1 GiB device-to-device copy (bench.py --copy-calibration) under "
                          "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE",
           "traffic_scope": "L2 egress: FETCH_SIZE x scale + WRITE_SIZE x scale; includes "
                            "Infinity Cache hits (this GPU exposes no MALL hit counter)",
           "kernels": kernels}
    # the bench line of the traced run names the tuning: per-run bytes of its
    # level-blocked kernel and of the p x SpMV kernel, keyed as bench.py looks
    # them up
    line = None
    for f in sorted(glob.glob(os.path.join(d, "trace*.log"))):
        with open(f) as fh:
            for ln in fh:
                if ln.startswith("{"):
                    line = json.loads(ln)
    if line is not None:
        with open(KERNEL_SRC, "rb") as fh:
            out["kernels_sha256"] = hashlib.sha256(fh.read()).hexdigest()
        out["command"] = line.get("command")
        out["workload"] = line.get("config", {}).get("workload", line.get("workload", ""))
    if line is not None and "roofline" in line:
        p = line["config"]["p"]

        def run_entry(pred, launches):
            ks = [k for k in kernels if pred(k.split("::")[-1]) and
                  "l2_egress_bytes_per_launch" in kernels[k]]
            if not ks:
                return None
            k = max(ks, key=lambda k: kernels[k]["launches"] * kernels[k]["avg_us"])
            e = kernels[k]
            return {"kernel": k, "launches_per_run": launches, "avg_launch_us": e["avg_us"],
                    "l2_egress_bytes_per_run": e["l2_egress_bytes_per_launch"] * launches,
                    "l2_hit_rate": e.get("l2_hit_rate")}

        runs = {}
        lbk = line["roofline"].get("run_key")
        lbe = run_entry(lambda k: k.startswith(("lb_", "xcd_", "step_")),
                        line["plan"]["launches_per_run"])
        if lbk and lbe:
            runs[lbk] = lbe
        be = run_entry(lambda k: k.startswith("spmv_"), p)
        if be:
            runs["pxspmv:" + line["baseline_pxspmv"]["reorder"]] = be
        out["runs"] = runs
    return out


def counters_markdown(dirs, summary):
    """Markdown summary of a reduced profile: the commands that made it,
    the --stats table (first directory) and the per-run traffic of the two
    kernels (every directory)."""
    import csv
    import glob
    d = dirs[0]
    cmds = summary.get("commands") or [summary.get("command")]
    lines = [f"# Kernel trace and L2-egress traffic: {summary.get('workload', '')}", "",
             "Commands (from the repository root on one MI355X, after "
             "`cd /tmp && export TMPDIR=/tmp`; `bench.py` by its full path):", "", "```"]
    for rel, cmd in zip(dirs, cmds):
        cmd = cmd or "python3 bench.py ..."
        for sub, opt in (("trace", "--kernel-trace --stats"),
                         ("fetch", "--pmc FETCH_SIZE --kernel-trace"),
                         ("write", "--pmc WRITE_SIZE --kernel-trace"),
                         ("tcc", "--pmc TCC_HIT_sum TCC_MISS_sum --kernel-trace")):
            lines.append(f"rocprofv3 {opt} -d {rel}/{sub} -o run --output-format csv -- {cmd}")
    for sub, c in (("cfetch", "FETCH_SIZE"), ("cwrite", "WRITE_SIZE")):
        lines.append(f"rocprofv3 --pmc {c} --kernel-trace -d {d}/{sub} -o copy --output-format csv "
                     f"-- python3 bench.py --copy-calibration")
    lines += [f"python3 bench.py --reduce-counters {' '.join(dirs)} > summary.json",
              f"python3 bench.py --reduce-counters {' '.join(dirs)} --markdown > summary.md",
              "```", "",
              f"kernels.hip SHA-256: `{summary.get('kernels_sha256')}`", "",
              "## --stats summary (kernel_stats.csv, the 12 longest in total)", "",
              "| Kernel | Calls | Average µs | Total ms |", "|---|---|---|---|"]
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "trace", "**", "*kernel_stats.csv"), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows[:12]:
        lines.append(f"| `{_kernel_key(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['TotalDurationNs']) / 1e6:.2f} |")
    lines += ["", "## Traffic per run", "",
              f"Scope: {summary.get('traffic_scope')}.  Calibration: {summary.get('calibration')}; "
              f"FETCH_SIZE scale {summary.get('fetch_scale')}, WRITE_SIZE scale "
              f"{summary.get('write_scale')}.", "",
              "| Run | Kernel | Launches/run | Avg launch µs | L2-egress bytes/run | L2 hit rate |",
              "|---|---|---|---|---|---|"]
    for key, e in summary.get("runs", {}).items():
        lines.append(f"| `{key}` | `{e['kernel']}` | {e['launches_per_run']} | {e['avg_launch_us']} | "
                     f"{e['l2_egress_bytes_per_run']:,} | {e.get('l2_hit_rate')} |")
    lines += ["", "## Traffic per launch of the MPK kernels", "",
              "| Kernel | Launches | Avg µs | L2-egress bytes/launch | L2 hit rate |",
              "|---|---|---|---|---|"]
    hot = ("lb_", "spmv_", "step_", "xcd_", "combine_")
    for k, e in sorted(summary.get("kernels", {}).items(), key=lambda kv: -kv[1]["avg_us"] *
                       kv[1]["launches"]):
        if k.split("::")[-1].startswith(hot) and "l2_egress_bytes_per_launch" in e:
            lines.append(f"| `{k}` | {e['launches']} | {e['avg_us']} | "
                         f"{e['l2_egress_bytes_per_launch']:,} | {e.get('l2_hit_rate')} |")
    return "\n".join(lines) + "\n"


def sweep_markdown(sweep):
    """Markdown table of a --bandwidth-sweep result."""
    lines = ["| Working set | global GB/s | xcd_local GB/s |", "|---|---|---|"]
    by = {}
    for r in sweep["points"]:
        by.setdefault(r["bytes"], {})[r["mode"]] = r["GBs"]
    for b in sorted(by):
        size = f"{b >> 20} MiB" if b < (1 << 30) else f"{b >> 30} GiB"
        lines.append(f"| {size} | {by[b].get('global', '')} | {by[b].get('xcd_local', '')} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving session")
    ap.add_argument("--serve-rate", default="190,250",
                    help="Poisson arrival rates (requests/s, comma-separated) of the paced "
                         "serving passes; the first is the headline")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the banded and Anderson workloads")
    ap.add_argument("--schedule", default=None,
                    help="run this level-blocked schedule instead of autotuning (profiling)")
    ap.add_argument("--chunk", type=int, default=16384, help="chunk nonzeros with --schedule")
    ap.add_argument("--cache-mib", type=int, default=64, help="cache budget with --schedule")
    ap.add_argument("--lag", type=int, default=0, help="wavefront lag with --schedule")
    ap.add_argument("--workgroups", type=int, default=0,
                    help="persistent workgroups with --schedule (0: the library's default)")
    ap.add_argument("--seg-powers", type=int, default=0,
                    help="powers per launch with --schedule (0: all)")
    ap.add_argument("--dynamic-tickets", type=int, default=0, choices=[0, 1],
                    help="with --schedule: 1 = tasks from a shared counter, 0 = static order")
    ap.add_argument("--reorder", default="bfs", choices=["bfs", "none", "sublevels"],
                    help="level construction with --schedule")
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(WORKLOAD_TEXT),
                    help="headline workload (default: the 128^3 stencil; others for profiling)")
    ap.add_argument("--value-bits", type=int, default=None, choices=[32, 64],
                    help="matrix value precision (default: the workload's)")
    ap.add_argument("--time-step-only", action="store_true",
                    help="print only the Chebyshev time-step measurement (for profiling)")
    ap.add_argument("--bandwidth-sweep", action="store_true",
                    help="only run the load-bandwidth probe over 1 MiB .. 4 GiB working sets")
    ap.add_argument("--reduce-counters", metavar="DIR", nargs="+", default=None,
                    help="reduce the rocprofv3 output of a profiled configuration (DIR/trace, "
                         "fetch, write, tcc, cfetch, cwrite) to JSON on stdout and stop")
    ap.add_argument("--markdown", action="store_true",
                    help="with --reduce-counters: print the markdown summary instead of JSON")
    ap.add_argument("--sweep-markdown", metavar="JSON", default=None,
                    help="print a --bandwidth-sweep result file as a markdown table and stop")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three 1 GiB device-to-device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); sharding the kernel over "
              "several GPUs is a design note, not a benchmark here.", file=sys.stderr)
        sys.exit(2)

    if args.reduce_counters:
        red = reduce_counter_dirs(args.reduce_counters)
        if args.markdown:
            print(counters_markdown(args.reduce_counters, red), end="", flush=True)
        else:
            print(json.dumps(red, indent=1), flush=True)
        return
    if args.sweep_markdown:
        with open(args.sweep_markdown) as f:
            print(sweep_markdown(json.load(f)), end="", flush=True)
        return

    if not args.no_serve and not (args.time_step_only or args.bandwidth_sweep or
                                  args.copy_calibration):
        # The serving session runs one stream per pool matrix beside the
        # default stream.  HIP maps streams onto GPU_MAX_HW_QUEUES hardware
        # queues (4 unless set), and streams that share a queue run in its
        # order: a short batch then waits for a long one queued before it
        # (measured: 0.1 ms alone, 62 ms behind two long batches).  The
        # setting is read when HIP starts, so it is made before torch uses
        # the device.
        if int(os.environ.get("GPU_MAX_HW_QUEUES") or 4) < SERVE_HW_QUEUES:
            os.environ["GPU_MAX_HW_QUEUES"] = str(SERVE_HW_QUEUES)
    import torch
    import paper_2405_12525_amd as mpk
    import workloads as w

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": a.numel() * 8, "copies": 3}), flush=True)
        return
    if args.bandwidth_sweep:
        print(json.dumps(bandwidth_sweep(torch, mpk, stream)), flush=True)
        return
    if args.time_step_only:
        fixed = None
        if args.schedule is not None:
            fixed = dict(schedule=args.schedule, chunk_nnz=args.chunk, lag=args.lag,
                         workgroups=args.workgroups, seg_powers=args.seg_powers,
                         cache_bytes=args.cache_mib << 20, dynamic_tickets=args.dynamic_tickets)
        ts = time_step(torch, mpk, w, args.steps, args.warmup, stream, not args.no_cpu, fixed)
        ts["command"] = "python3 bench.py " + " ".join(sys.argv[1:])
        ts["workload"] = ("Chebyshev time step, Anderson 160^3 periodic, FP32 values, 4 complex "
                          "states, M = 16, dt = 1")
        print(json.dumps(ts), flush=True)
        return
    t0 = time.perf_counter()
    A, x, p, kind = w.config(args.workload)
    text, default_vb = WORKLOAD_TEXT[args.workload]
    vb = args.value_bits or default_vb
    cheb = kind == "chebyshev"
    coefs = mpk.chebyshev_coefficients(p) if cheb else None
    R = x.shape[1]
    log(f"[bench] generated {args.workload}: n={A.n} nnz={A.nnz} in {time.perf_counter() - t0:.1f}s")
    xd = torch.from_numpy(x).cuda()
    Y = torch.empty((p, A.n, R), dtype=torch.float64, device="cuda")
    B = torch.empty_like(Y)
    flop = mpk.flops(A.nnz, A.n, p, R, recur=cheb)

    def run_lb(P, out):
        return (P.run_recur(xd, *coefs, Y=out, stream=stream) if cheb
                else P.run(xd, p, out, stream=stream))

    def run_base(P, out):
        return (P.run_baseline_recur(xd, *coefs, Y=out, stream=stream) if cheb
                else P.run_baseline(xd, p, out, stream=stream))

    # p x SpMV baseline: best of BFS and original order
    base = {}
    for ro in (("bfs", "none") if args.schedule is None else (args.reorder,)):
        P = mpk.Plan(A, reorder=ro, value_bits=vb)
        base[ro] = time_calls(lambda: run_base(P, B), args.steps, args.warmup, torch, stream)
        log(f"[bench] p x SpMV reorder={ro}: {base[ro]['median_ms']:.3f} ms "
            f"({flop / base[ro]['median_ms'] / 1e6:.1f} Gflop/s)")
        P.close()
    best_base = min(base, key=lambda r: base[r]["median_ms"])

    # level-blocked run: the autotuner's choice in each order, the fastest one reported
    lb = None
    by_order = {}
    for ro in (("bfs", "none", "sublevels") if args.schedule is None else (args.reorder,)):
        t0 = time.perf_counter()
        Q = mpk.Plan(A, reorder=ro, value_bits=vb)
        if args.schedule is None:
            tq = Q.autotune(xd, p, Y, reps=3, recur=cheb, stream=stream)
        else:
            tq = Q.tune(schedule=args.schedule, chunk_nnz=args.chunk,
                        cache_bytes=args.cache_mib << 20, lag=args.lag,
                        workgroups=args.workgroups, seg_powers=args.seg_powers,
                        dynamic_tickets=args.dynamic_tickets)
        r = time_calls(lambda: run_lb(Q, Y), args.steps, args.warmup, torch, stream)
        Q.sync()
        log(f"[bench] level-blocked reorder={ro}: autotuned in {time.perf_counter() - t0:.1f}s "
            f"-> {tq['schedule']} C={tq['cache_bytes'] >> 20} MiB chunk={tq['chunk_nnz']}: "
            f"{r['median_ms']:.3f} ms ({flop / r['median_ms'] / 1e6:.1f} Gflop/s)")
        by_order[ro] = {"ms": round(r["median_ms"], 4), "schedule": tq["schedule"],
                        "chunk_nnz": tq["chunk_nnz"], "workgroups": tq["workgroups"]}
        if ro == "sublevels" and args.schedule is None:
            # the XCD schedule on the sub-level order: each XCD's part of
            # every level is a run of sub-levels
            Q.tune(schedule="xcd", chunk_nnz=16384, lag=0, workgroups=0)
            rx = time_calls(lambda: run_lb(Q, Y), args.steps, args.warmup, torch, stream)
            Q.sync()
            sx = Q.schedule(p)
            inf = Q.info()
            by_order["sublevels_xcd"] = {"ms": round(rx["median_ms"], 4), "schedule": "xcd",
                                         "chunk_nnz": 16384, "lag": sx["lag"],
                                         "window_bytes": int(sx["window_bytes"]),
                                         "max_sublevels": inf["max_sublevels"]}
            log(f"[bench] sub-level order, XCD schedule: {rx['median_ms']:.3f} ms")
            Q.tune(**{k: v for k, v in tq.items() if k != "ms"})
        if lb is None or r["median_ms"] < lb["median_ms"]:
            if lb is not None:
                P.close()
            lb, P, tune, reorder = r, Q, tq, ro
        else:
            Q.close()
    info = P.info()
    sched = P.schedule(p)
    # the same plan from a CSR already in device memory (mpk_plan_device)
    import types
    dcsr = types.SimpleNamespace(n=A.n, rowptr=torch.from_numpy(A.rowptr).cuda(),
                                 col=torch.from_numpy(A.col).cuda(),
                                 val=torch.from_numpy(A.val).cuda())
    dev_ms = {}
    for ro in ("none", "bfs"):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Pd = mpk.Plan(dcsr, reorder=ro, value_bits=vb)
            ts.append((time.perf_counter() - t0) * 1e3)
            Pd.close()
        dev_ms[ro] = round(statistics.median(ts), 1)
    del dcsr
    log(f"[bench] plans from a device CSR: {dev_ms} ms")
    run_base(P, B)
    run_lb(P, Y)
    stream.synchronize()
    P.sync()
    same = bool(torch.equal(Y, B))
    log(f"[bench] level-blocked bit-identical to p x SpMV: {same}")
    # the same run captured in a HIP graph and replayed
    G = P.capture(xd, p, Y, *(coefs if cheb else ()))
    gr = time_calls(lambda: G.launch(stream=stream), args.steps, args.warmup, torch, stream)
    stream.synchronize()
    graph_same = bool(torch.equal(Y, B))
    G.close()
    log(f"[bench] HIP graph replay: {gr['median_ms']:.3f} ms, equal: {graph_same}")

    Yh = None if args.no_cpu else Y.cpu().numpy()   # for the per-power check on the CPU leg
    extra = (p - 1) * 8 * A.n * R if cheb else 0  # y_{k-1} read again by the recurrence
    lb_bytes = algorithmic_bytes(A.n, A.nnz, p, R, vb // 8, "lb", A.n if reorder != "none" else 0)
    trad_bytes = algorithmic_bytes(A.n, A.nnz, p, R, vb // 8, "trad",
                                   A.n if best_base == "bfs" else 0) + extra
    achieved = lb_bytes / (lb["mean_ms"] * 1e-3) / 1e9
    effective = trad_bytes / (lb["mean_ms"] * 1e-3) / 1e9
    run_key = "level_blocked:{schedule}:{chunk_nnz}:{cm}:{lag}:{workgroups}:{ro}".format(
        cm=tune["cache_bytes"] >> 20, ro=reorder, **tune)
    value = flop / (lb["median_ms"] * 1e-3) / 1e9
    bmed = base[best_base]["median_ms"]
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Gflop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(lb["median_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if vb == 64 else "f64 (f32-stored values)",
        "data": "synthetic",
        "config": {"workload": text.format(vb="FP64" if vb == 64 else "FP32-value"),
                   "n": A.n, "nnz": A.nnz, "p": p, "nrhs": R, "reorder": reorder,
                   "schedule": tune["schedule"], "cache_mib": tune["cache_bytes"] >> 20,
                   "chunk_nnz": tune["chunk_nnz"], "lag": sched["lag"],
                   "workgroups": tune["workgroups"], "seg_powers": tune["seg_powers"],
                   "task_order": "shared counter" if tune["dynamic_tickets"] else "static",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, vb, run_key),
                     "traffic_scope": "L2 egress bytes per run: FETCH_SIZE x 2.0 + WRITE_SIZE x "
                                      "1.0 (copy-calibrated); Infinity Cache hits included",
                     "kernel": "level-blocked run (all launches of one mpk_run)",
                     "run_key": run_key,
                     "algorithmic_bytes": lb_bytes,
                     "effective_GBs_vs_pxspmv_traffic": round(effective, 1),
                     "effective_frac_vs_pxspmv_traffic": round(effective / HBM_PEAK_GBS, 4)},
        "baseline_pxspmv": {"gflops": round(flop / (bmed * 1e-3) / 1e9, 2), "ms": round(bmed, 4),
                            "reorder": best_base, "algorithmic_bytes": trad_bytes,
                            "achieved_GBs": round(trad_bytes / (base[best_base]["mean_ms"] * 1e-3)
                                                  / 1e9, 1),
                            "traffic": measured_traffic(args.workload, vb, "pxspmv:" + best_base)},
        "speedup_vs_pxspmv": round(bmed / lb["median_ms"], 3),
        "level_blocked_by_order": by_order,
        "hip_graph": {"ms": round(gr["median_ms"], 4), "bit_identical": graph_same,
                      "launches_per_run": sched["n_steps"]},
        "bit_identical_to_pxspmv": same,
        "plan": {"host_ms": round(info["plan_ms"], 1), "levels": info["n_levels"],
                 "chunks": sched["n_chunks"], "launches_per_run": sched["n_steps"],
                 "window_bytes": int(sched["window_bytes"]), "max_reach": sched["max_reach"],
                 "window_within_budget_C": bool(sched["window_bytes"] <= tune["cache_bytes"]),
                 "sliced_layout": bool(info["sliced_layout"]),
                 "sliced_col_bits": info["sliced_col_bits"],
                 "spmv_equivalents": round(info["plan_ms"] / (bmed / p), 1),
                 "from_device_csr_ms": dev_ms,
                 "from_device_csr_spmv_equivalents": {k: round(v / (bmed / p), 1)
                                                      for k, v in dev_ms.items()}},
    }
    if args.schedule is not None:
        out["command"] = "python3 bench.py " + " ".join(sys.argv[1:])
    P.close()
    del Y, B
    if not args.no_configs and args.schedule is None and args.workload == WORKLOAD:
        out["other_configs"] = other_configs(torch, mpk, w, args.steps, args.warmup, stream,
                                             not args.no_cpu)
        out["other_configs"]["cheb_time_step_anderson160_m16_s4_fp32"] = time_step(
            torch, mpk, w, args.steps, args.warmup, stream, not args.no_cpu)
    if not args.no_serve and args.workload == WORKLOAD:
        try:
            out["serving"] = serving(torch, mpk, w,
                                     [float(r) for r in args.serve_rate.split(",")])
        except mpk.MPKError as e:
            # a failed serving session is reported in the line, which still
            # carries the measured MPK runs above
            log(f"[bench] serving failed: {e}")
            out["serving"] = {"error": str(e)}
    if not args.no_cpu and args.workload == WORKLOAD:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"], ref = cpu_baseline(A, x, p)
        rel = per_power_rel_err(Yh, ref)
        out["parity_vs_fp64_oracle"] = {"rel_err_per_power": rel, "tolerance": 1e-12,
                                        "within_tolerance": max(rel) <= 1e-12}
        log(f"[bench] per-power relative error vs the FP64 oracle: max {max(rel):.2e}")
        del ref, Yh
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
