"""GPU tests of the runtime around the kernels: the autotuner and captured
HIP graphs (every replay checked against the eager run and the oracle)."""
import time

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mpk = pytest.importorskip("paper_2405_12525_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("sched", ["wave", "steps", "xcd"])
def test_prepare_then_run_is_exact(sched):
    """Runs after mpk_plan_prepare (schedules and slice tables built ahead,
    the slice tables shared by every R >= 4) equal the oracle bit for bit,
    as do runs on a plan that builds them lazily."""
    A = w.stencil_3d27(14)
    P = mpk.Plan(A)
    Q = mpk.Plan(A)
    for plan in (P, Q):
        plan.tune(schedule=sched, chunk_nnz=3000)
    P.prepare(range(1, 7))        # every R in 1..16
    g = np.random.default_rng(9)
    for p, R in [(1, 1), (5, 3), (6, 16), (4, 7), (6, 4)]:
        x = dev(g.uniform(-1, 1, (A.n, R)))
        ref = oracle.powers(A, host(x), p)
        assert np.array_equal(host(P.run(x, p)), ref), (p, R)
        assert np.array_equal(host(Q.run(x, p)), ref), (p, R)
        assert np.array_equal(host(P.run_baseline(x, p)), ref), (p, R)
    # p above the segment length: every segment's schedule is prepared
    P.tune(schedule=sched, chunk_nnz=3000, seg_powers=3)
    P.prepare(7, 2)
    x = dev(g.uniform(-1, 1, (A.n, 2)))
    assert np.array_equal(host(P.run(x, 7)), oracle.powers(A, host(x), 7))
    with pytest.raises(mpk.MPKError):
        P.prepare(0, 1)
    with pytest.raises(mpk.MPKError):
        P.prepare(3, 17)
    P.close()
    Q.close()


@pytest.mark.parametrize("sched", ["wave", "steps"])
def test_prepare_allows_stream_capture_without_a_run(sched):
    """After mpk_plan_prepare alone, mpk_run can be captured into the
    caller's own graph; every replay equals the oracle.  Without it the
    capture is refused with a clear error instead of planning inside it."""
    A = w.stencil_3d27(12)
    P = mpk.Plan(A)
    P.tune(schedule=sched, chunk_nnz=3000)
    x = dev(np.random.default_rng(4).uniform(-1, 1, (A.n, 2)))
    Y = torch.empty((5, A.n, 2), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    P.prepare(3, 2)      # another p: the refused capture below launches nothing
    torch.cuda.synchronize()
    with pytest.raises(mpk.MPKError, match="mpk_plan_prepare"):
        g0 = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g0, stream=s):
            P.run(x, 5, Y=Y, stream=s)
    torch.cuda.synchronize()
    P.prepare(5, 2)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        P.run(x, 5, Y=Y, stream=s)
    torch.cuda.synchronize()
    ref = oracle.powers(A, host(x), 5)
    for _ in range(3):
        Y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(Y), ref)
    del g
    P.close()


def test_autotune_choice_is_exact_and_cached():
    A = w.stencil_3d27(32)
    x = w.uniform_vectors(A.n, 2, 11)
    xd = dev(x)
    P = mpk.Plan(A)
    t = P.autotune(xd, 5, reps=2, force=True)
    assert t["schedule"] in ("steps", "wave", "xcd", "powers") and t["ms"] > 0
    Y = P.run(xd, 5)
    P.sync()
    assert np.array_equal(host(Y), oracle.powers(A, x, 5))
    # a second plan of the same matrix finds the cached choice without timing
    Q = mpk.Plan(A)
    t0 = time.perf_counter()
    t2 = Q.autotune(xd, 5)
    assert time.perf_counter() - t0 < 0.5
    tuned = ("schedule", "cache_bytes", "chunk_nnz", "lag", "workgroups", "seg_powers",
             "skip_ahead", "dynamic_tickets")
    assert {k: t2[k] for k in tuned} == {k: t[k] for k in tuned}
    # a plan set to the shared counter keeps it in every candidate, and its
    # choice is cached apart from the fixed-order one
    Q.tune(dynamic_tickets=1)
    t3 = Q.autotune(xd, 5, reps=1, force=True)
    assert t3["dynamic_tickets"] == 1 and Q.tuning["dynamic_tickets"] == 1
    Y3 = Q.run(xd, 5)
    Q.sync()
    assert np.array_equal(host(Y3), oracle.powers(A, x, 5))
    R = mpk.Plan(A)
    R.tune(dynamic_tickets=1)
    t4 = R.autotune(xd, 5)
    assert {k: t4[k] for k in tuned} == {k: t3[k] for k in tuned}
    P.close()
    Q.close()
    R.close()


def test_autotune_recurrence_fp32():
    A = w.anderson_3d(16)
    x = w.random_sign_unit_vectors(A.n, 8, 3)
    xd = dev(x)
    P = mpk.Plan(A, value_bits=32)
    P.autotune(xd, 6, reps=1, recur=True, force=True)
    al, be, ga = mpk.chebyshev_coefficients(6)
    Y = P.run_recur(xd, al, be, ga)
    P.sync()
    ref = oracle.recur(A, x, al, be, ga, value_bits=32)
    assert np.array_equal(host(Y), ref)
    P.close()


@pytest.mark.parametrize("sched", ["steps", "wave", "xcd"])
def test_graph_replays_match_eager(sched):
    A = w.stencil_3d27(24)
    x = w.uniform_vectors(A.n, 1, 21)
    xd = dev(x)
    P = mpk.Plan(A)
    P.tune(schedule=sched, chunk_nnz=2000)
    eager = host(P.run(xd, 6))
    assert np.array_equal(eager, oracle.powers(A, x, 6))
    Yg = torch.empty((6, A.n, 1), dtype=torch.float64, device="cuda")
    G = P.capture(xd, 6, Yg)
    s = torch.cuda.Stream()
    for i in range(4):
        Yg.fill_(np.nan)
        torch.cuda.synchronize()
        G.launch(stream=s)
        s.synchronize()
        assert np.array_equal(host(Yg), eager), f"replay {i}"
        # unrelated eager work on the same plan between replays
        other = P.run(dev(w.uniform_vectors(A.n, 1, 100 + i)), 3)
        P.sync()
        del other
    G.close()
    P.sync()
    P.close()


def test_graph_recurrence_replays():
    A = w.anderson_3d(12)
    x = w.random_sign_unit_vectors(A.n, 4, 8)
    xd = dev(x)
    P = mpk.Plan(A)
    al, be, ga = mpk.chebyshev_coefficients(8)
    ref = oracle.recur(A, x, al, be, ga)
    Yg = torch.empty((8, A.n, 4), dtype=torch.float64, device="cuda")
    G = P.capture(xd, 8, Yg, al, be, ga)
    for _ in range(3):
        Yg.zero_()
        G.launch()
        assert np.array_equal(host(Yg), ref)
    G.close()
    P.close()


def test_torch_allocator_hook():
    mpk.use_torch_allocator(True)
    try:
        before = dict(mpk.allocator_stats)
        A = w.stencil_3d27(20)
        x = w.uniform_vectors(A.n, 2, 5)
        P = mpk.Plan(A)
        P.tune(schedule="wave", chunk_nnz=3000)
        Y = P.run(dev(x), 4)
        P.sync()
        assert np.array_equal(host(Y), oracle.powers(A, x, 4))
        used = mpk.allocator_stats["allocs"] - before["allocs"]
        assert used >= 4  # matrix arrays, slices, schedule, workspace
        P.close()
        torch.cuda.synchronize()
        assert mpk.allocator_stats["frees"] - before["frees"] == used
    finally:
        mpk.use_torch_allocator(False)
    # plans made afterwards use hipMalloc again
    n0 = mpk.allocator_stats["allocs"]
    Q = mpk.Plan(w.stencil_2d5(10))
    Q.close()
    assert mpk.allocator_stats["allocs"] == n0


def test_load_probe_sums_exactly():
    n = 1 << 20
    buf = torch.arange(n, dtype=torch.float64, device="cuda") % 7   # small integers: exact sums
    sink = mpk.probe_load(buf, passes=3, workgroups=512)
    torch.cuda.synchronize()
    assert sink.shape == (512,)
    assert float(sink.sum().item()) == 3 * float(buf.sum().item())
