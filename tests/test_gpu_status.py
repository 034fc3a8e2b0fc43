"""GPU: per-run failure status, runs that read their inputs without cache
invalidation, and the XCD schedule's progress under concurrent launches.

* A run abandoned because a dependency wait hit its limit (forced from the
  host with a 1 us limit; every kernel still exits normally) reports 1
  through mpk_run_status on its stream, and mpk_plan_sync reports it once.
  The next run on the same plan starts clean: status 0 and exact results.
* Level-blocked runs whose chunks own whole 128-byte lines of the outputs
  read their inputs without invalidating caches first; repeated runs with
  different inputs into the same output buffer must still equal the p x SpMV
  baseline bit for bit (no stale line survives from a previous run or from a
  line read before it was complete), in every row order and for ragged
  sizes where the library falls back to invalidation.
* Two XCD-schedule runs and other persistent runs in flight together on
  separate streams all complete with exact results.
"""
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


def dev_x(n, R, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.uniform(-1, 1, size=(n, R))).cuda()


def status_of(P, stream=None):
    out = torch.zeros(1, dtype=torch.int32, pin_memory=True)
    P.run_status(out, stream=stream)
    torch.cuda.synchronize()
    return int(out[0])


def test_status_is_zero_after_good_runs():
    A = w.stencil_3d27(12)
    P = mpk.Plan(A)
    x = dev_x(A.n, 2, 1)
    Y = P.run(x, 5)
    assert status_of(P) == 0
    P.sync()
    assert np.array_equal(Y.cpu().numpy(), oracle.powers(A, x.cpu().numpy(), 5))
    P.close()


def test_timed_out_run_is_reported_and_does_not_poison_the_next():
    A = w.stencil_3d27(40)
    P = mpk.Plan(A, reorder="none")
    x = dev_x(A.n, 1, 2)
    ref = oracle.powers(A, x.cpu().numpy(), 8)
    # many small chunks, the smallest slack and a 1 us wait limit: waits fail
    P.tune(schedule="wave", chunk_nnz=1024, lag=1, spin_limit_us=1)
    stream = torch.cuda.Stream()
    Y = torch.empty((8, A.n, 1), dtype=torch.float64, device="cuda")
    P.run(x, 8, Y, stream=stream)
    first = status_of(P, stream)
    with pytest.raises(mpk.MPKError) if first else _nullcontext():
        P.sync()
    if not first:   # no wait failed after all: then the result must be exact
        assert np.array_equal(Y.cpu().numpy(), ref)
    # the same plan, the same workspace, a normal limit: clean and exact
    P.tune(schedule="wave", chunk_nnz=1024, lag=1, spin_limit_us=0)
    P.run(x, 8, Y, stream=stream)
    assert status_of(P, stream) == 0
    P.sync()
    assert np.array_equal(Y.cpu().numpy(), ref)
    assert first == 1, "the 1 us limit was expected to abandon the first run"
    P.close()


class _nullcontext:
    def __enter__(self):
        return None

    def __exit__(self, *a):
        return False


@pytest.mark.parametrize("order,reorder,n_side,R", [
    ("original", "none", 24, 1),    # n = 13824: n*R multiple of 16, no invalidation
    ("original", "none", 24, 3),
    ("plan", "bfs", 24, 2),         # plan order: outputs in plan rows, no invalidation
    ("original", "bfs", 24, 1),     # caller's order through a permutation: invalidation
    ("original", "none", 23, 1),    # n = 12167: ragged, invalidation
    ("original", "none", 23, 16),   # n*R multiple of 16 again
])
@pytest.mark.parametrize("sched", ["wave", "powers"])
def test_runs_without_invalidation_equal_baseline_on_reused_outputs(order, reorder, n_side, R,
                                                                    sched):
    A = w.stencil_3d27(n_side)
    P = mpk.Plan(A, reorder=reorder, order=order)
    P.tune(schedule=sched, chunk_nnz=700, lag=2)
    p = 6
    Y = torch.empty((p, A.n, R), dtype=torch.float64, device="cuda")
    B = torch.empty_like(Y)
    for seed in range(4):
        x = dev_x(A.n, R, 100 + seed)
        if order == "plan":
            x = P.permute(x, to_plan=True)
        P.run(x, p, Y)
        P.run_baseline(x, p, B)
        P.sync()
        assert torch.equal(Y, B), (seed, order, reorder, n_side, R, sched)
    # the last one against the oracle too
    xo = x if order == "original" else P.permute(x, to_plan=False)
    ref = oracle.powers(A, xo.cpu().numpy(), p)
    got = Y if order == "original" else P.permute(Y.reshape(p, A.n, R), to_plan=False)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().reshape(ref.shape), ref)
    P.close()


def test_concurrent_xcd_and_wave_runs_complete():
    mats = [w.anderson_3d(10), w.stencil_3d27(16), w.anderson_3d(12)]
    plans = [mpk.Plan(A) for A in mats]
    plans[0].tune(schedule="xcd", chunk_nnz=500)
    plans[1].tune(schedule="wave", chunk_nnz=1500)
    plans[2].tune(schedule="xcd", chunk_nnz=800)
    streams = [torch.cuda.Stream() for _ in range(4)]
    jobs = []
    for rep in range(6):
        for i, (A, P) in enumerate(zip(mats, plans)):
            s = streams[(rep + i) % len(streams)]
            x = dev_x(A.n, 1 + (rep % 3), 10 * rep + i)
            Y = torch.empty((5, A.n, x.shape[1]), dtype=torch.float64, device="cuda")
            with torch.cuda.stream(s):
                P.run(x, 5, Y, stream=s)
            jobs.append((A, P, x, Y, s))
    for P, s in {(P, s) for _, P, _, _, s in jobs}:
        assert status_of(P, s) == 0
    torch.cuda.synchronize()
    for P in plans:
        P.sync()
    for A, P, x, Y, _ in jobs:
        assert np.array_equal(Y.cpu().numpy(), oracle.powers(A, x.cpu().numpy(), 5))
    for P in plans:
        P.close()


def test_static_and_dynamic_task_orders_agree_and_overlap_safely():
    """The static task order (every workgroup takes every W-th ticket) and
    the shared counter give the same bits; static-order launches of several
    plans on several streams, mixed with XCD, dynamic and per-diagonal
    launches, all complete (the device gate orders the ones that need the
    device alone) and match the oracle."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    mats = [w.stencil_3d27(18), w.anderson_3d(12), w.stencil_2d5(90), w.stencil_3d27(14)]
    plans = [mpk.Plan(A) for A in mats]
    plans[0].tune(schedule="powers", chunk_nnz=2000, workgroups=8 * cus)
    plans[1].tune(schedule="wave", chunk_nnz=1500, workgroups=2 * cus, lag=40)
    plans[2].tune(schedule="xcd", chunk_nnz=800)
    plans[3].tune(schedule="wave", chunk_nnz=1200, dynamic_tickets=1)
    # same bits with either order on one plan
    x = dev_x(mats[0].n, 3, 77)
    Ys = plans[0].run(x, 6)
    plans[0].tune(dynamic_tickets=1)
    Yd = plans[0].run(x, 6)
    torch.cuda.synchronize()
    plans[0].sync()
    assert torch.equal(Ys, Yd)
    plans[0].tune(dynamic_tickets=0)
    streams = [torch.cuda.Stream() for _ in range(3)]
    jobs = []
    for rep in range(5):
        for i, (A, P) in enumerate(zip(mats, plans)):
            s = streams[(rep + i) % len(streams)]
            x = dev_x(A.n, 1 + (rep % 4), 100 * rep + i)
            Y = torch.empty((6, A.n, x.shape[1]), dtype=torch.float64, device="cuda")
            with torch.cuda.stream(s):
                P.run(x, 6, Y, stream=s)
            jobs.append((A, P, x, Y, s))
    torch.cuda.synchronize()
    for P, s in {(P, s) for _, P, _, _, s in jobs}:
        assert status_of(P, s) == 0
    for P in plans:
        P.sync()
    for A, P, x, Y, _ in jobs:
        assert np.array_equal(Y.cpu().numpy(), oracle.powers(A, x.cpu().numpy(), 6))
    for P in plans:
        P.close()


def test_captured_static_order_runs_overlap_safely_with_eager_runs():
    """Graphs captured with the static task order are gated at launch: two
    graphs replayed on two streams next to eager static-order runs of
    another plan all complete, every replay equal to the oracle."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    A, B = w.stencil_3d27(16), w.anderson_3d(11)
    PA, PB = mpk.Plan(A), mpk.Plan(B)
    PA.tune(schedule="wave", chunk_nnz=1500, workgroups=4 * cus, lag=30)
    PB.tune(schedule="powers", chunk_nnz=1000, workgroups=8 * cus)
    xa = [dev_x(A.n, 2, 500 + i) for i in range(2)]
    Ya = [torch.empty((5, A.n, 2), dtype=torch.float64, device="cuda") for _ in range(2)]
    graphs = [PA.capture(xa[i], 5, Ya[i]) for i in range(2)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    xb = dev_x(B.n, 3, 600)
    refs_a = [oracle.powers(A, xa[i].cpu().numpy(), 5) for i in range(2)]
    ref_b = oracle.powers(B, xb.cpu().numpy(), 7)
    for rep in range(4):
        for i, G in enumerate(graphs):
            G.launch(stream=streams[i])
        Yb = PB.run(xb, 7, stream=streams[2])
        torch.cuda.synchronize()
        for i in range(2):
            assert np.array_equal(Ya[i].cpu().numpy(), refs_a[i]), (rep, i)
        assert np.array_equal(Yb.cpu().numpy(), ref_b), rep
    PA.sync()
    PB.sync()
    for G in graphs:
        G.close()
    PA.close()
    PB.close()
