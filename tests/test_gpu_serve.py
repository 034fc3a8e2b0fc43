"""GPU: continuous batching returns, for every request, exactly what the
request gives when run alone (bit for bit), and reports sane latencies."""
import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mpk = pytest.importorskip("paper_2405_12525_amd")
from paper_2405_12525_amd import serve  # noqa: E402


def device_x(n, R, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return (torch.rand((n, R), generator=g, device="cuda", dtype=torch.float64) * 2 - 1)


@pytest.mark.parametrize("realtime", [False, True])
def test_mix_equals_alone(realtime):
    torch.cuda.set_device(0)
    mats = [w.stencil_2d5(40), w.stencil_3d27(14), w.anderson_3d(10)]
    plans = [mpk.Plan(A) for A in mats]
    plans[1].tune(schedule="wave", chunk_nnz=3000)
    plans[2].tune(schedule="xcd", chunk_nnz=2000)
    specs = w.serving_requests(60, rate_per_s=4000.0, seed=77, pool_size=3, p_range=(1, 9),
                               rhs_choices=(1, 2, 3, 4, 8, 16))
    reqs = []
    for s in specs:
        kind = "chebyshev" if s["id"] % 5 == 0 else "powers"
        reqs.append(serve.Request(id=s["id"], arrival=s["t"], matrix=s["matrix"], p=s["p"],
                                  x=device_x(mats[s["matrix"]].n, s["R"], s["x_seed"]),
                                  kind=kind))
    srv = serve.Server(plans, n_streams=3, mem_budget=64 << 20)
    # level-blocked plans run beside other batches: tasks from the shared counter
    assert all(P.tuning["dynamic_tickets"] == 1 for P in plans)
    assert plans[2].tuning["schedule"] == "xcd" and plans[1].tuning["chunk_nnz"] == 3000
    res = srv.serve(reqs, realtime=realtime)
    assert [r.id for r in res] == [q.id for q in reqs]
    assert max(r.batch_size for r in res) > 1          # batching happened
    for q, r in zip(reqs, res):
        P = plans[q.matrix]
        if q.kind == "chebyshev":
            alone = P.run_recur(q.x, *mpk.chebyshev_coefficients(q.p))
        else:
            alone = P.run(q.x, q.p)
        torch.cuda.synchronize()
        assert r.Y.shape == alone.shape
        assert torch.equal(r.Y, alone), q.id
        assert r.done >= r.start >= 0 and r.latency >= 0
    # and against the oracle for a few
    for q, r in list(zip(reqs, res))[:6]:
        x = q.x.cpu().numpy()
        A = mats[q.matrix]
        ref = (oracle.recur(A, x, *mpk.chebyshev_coefficients(q.p)) if q.kind == "chebyshev"
               else oracle.powers(A, x, q.p))
        assert np.array_equal(r.Y.cpu().numpy(), ref)
    st = serve.summarize(res, reqs, plans)
    assert st["requests"] == 60 and st["p99_ms"] >= st["p50_ms"] > 0
    for P in plans:
        P.close()


def test_time_step_requests_equal_alone():
    torch.cuda.set_device(0)
    mats = [w.anderson_3d(12), w.stencil_3d27(12)]
    plans = [mpk.Plan(A) for A in mats]
    g = np.random.default_rng(5)
    reqs = []
    for i in range(24):
        m = i % 2
        kind = "time_step" if i % 3 else "powers"
        R = int(g.choice([2, 4])) if kind == "time_step" else int(g.choice([1, 2]))
        reqs.append(serve.Request(id=i, arrival=0.0005 * i, matrix=m,
                                  p=12 if kind == "time_step" else int(g.integers(2, 6)),
                                  x=device_x(mats[m].n, R, 300 + i), kind=kind,
                                  dt=(0.5 if i % 4 else 0.75) if kind == "time_step" else 0.0))
    srv = serve.Server(plans, n_streams=2, mem_budget=64 << 20)
    res = srv.serve(reqs, realtime=False)
    assert max(r.batch_size for q, r in zip(reqs, res) if q.kind == "time_step") > 1
    for q, r in zip(reqs, res):
        P = plans[q.matrix]
        alone = P.cheb_time_step(q.x, q.dt, q.p) if q.kind == "time_step" else P.run(q.x, q.p)
        torch.cuda.synchronize()
        assert r.Y.shape == alone.shape and torch.equal(r.Y, alone), q.id
    st = serve.summarize(res, reqs, plans)
    assert st["requests"] == 24 and st["gflops"] > 0
    for P in plans:
        P.close()


def test_unkept_outputs_equal_alone():
    """keep=False reuses one output and one staging buffer per stream; every
    output, seen through on_result before its buffer is reused, equals the
    request run alone, bit for bit, in a saturated and a paced pass."""
    torch.cuda.set_device(0)
    mats = [w.stencil_2d5(40), w.stencil_3d27(14), w.anderson_3d(10)]
    plans = [mpk.Plan(A) for A in mats]
    plans[2].tune(schedule="steps")
    specs = w.serving_requests(80, rate_per_s=4000.0, seed=91, pool_size=3, p_range=(1, 12),
                               rhs_choices=(1, 2, 3, 4, 8, 16))
    reqs = []
    for i, s in enumerate(specs):
        if i % 7 == 3 and s["R"] % 2 == 0:
            kind, p, dt = "time_step", 12, 0.5
        else:
            kind, p, dt = ("chebyshev" if i % 5 == 0 else "powers"), s["p"], 0.0
        reqs.append(serve.Request(id=s["id"], arrival=s["t"], matrix=s["matrix"], p=p,
                                  x=device_x(mats[s["matrix"]].n, s["R"], s["x_seed"]),
                                  kind=kind, dt=dt))
    assert {q.kind for q in reqs} == {"powers", "chebyshev", "time_step"}
    alone = {}
    for q in reqs:
        P = plans[q.matrix]
        if q.kind == "chebyshev":
            Y = P.run_recur(q.x, *mpk.chebyshev_coefficients(q.p))
        elif q.kind == "time_step":
            Y = P.cheb_time_step(q.x, q.dt, q.p)
        else:
            Y = P.run(q.x, q.p)
        alone[q.id] = Y.cpu().numpy()
    srv = serve.Server(plans, n_streams=3, mem_budget=64 << 20)
    got = {}

    def grab(q, Y):   # copy now: the buffer behind Y is reused by a later batch
        got[q.id] = Y.cpu().numpy()

    for realtime in (False, True):
        got.clear()
        res = srv.serve(reqs, realtime=realtime, keep=False, on_result=grab)
        assert all(r.Y is None for r in res)
        if not realtime:
            assert max(r.batch_size for r in res) > 1
        assert sorted(got) == sorted(q.id for q in reqs)
        for q in reqs:
            assert got[q.id].shape == alone[q.id].shape, q.id
            assert np.array_equal(got[q.id], alone[q.id]), (realtime, q.id, q.kind)
    for P in plans:
        P.close()


@pytest.mark.parametrize("inflight", [1, 3, "lanes"])
def test_baseline_plans_and_inflight_limit(inflight):
    """Plans served through the p x SpMV kernels (use_baseline) and the limit
    on batches in flight per matrix change neither result nor order: every
    output equals the request run alone through the level-blocked kernels, and
    the per-matrix summary covers every matrix."""
    torch.cuda.set_device(0)
    mats = [w.stencil_2d5(40), w.stencil_3d27(14), w.anderson_3d(10)]
    plans = [mpk.Plan(A) for A in mats]
    plans[1].tune(schedule="xcd", chunk_nnz=2000)
    specs = w.serving_requests(48, rate_per_s=4000.0, seed=123, pool_size=3, p_range=(1, 10),
                               rhs_choices=(1, 2, 4, 8))
    reqs = []
    for i, s in enumerate(specs):
        if i % 6 == 1 and s["R"] % 2 == 0:
            kind, p, dt = "time_step", 10, 0.5
        else:
            kind, p, dt = ("chebyshev" if i % 4 == 0 else "powers"), s["p"], 0.0
        reqs.append(serve.Request(id=s["id"], arrival=s["t"], matrix=s["matrix"], p=p,
                                  x=device_x(mats[s["matrix"]].n, s["R"], s["x_seed"]),
                                  kind=kind, dt=dt))
    if inflight == "lanes":
        srv = serve.Server(plans, n_streams=2, mem_budget=64 << 20, use_baseline=[True, False, True],
                           lanes=serve.Server.size_lanes(plans, 2))
    else:
        srv = serve.Server(plans, n_streams=3, mem_budget=64 << 20,
                           max_inflight_per_matrix=inflight, use_baseline=[True, False, True])
    # only the plan served through the level-blocked kernels is switched
    assert [P.tuning["dynamic_tickets"] for P in plans] == [0, 1, 0]
    srv.prepare(10)   # every shape these requests can form, built ahead
    res = srv.serve(reqs, realtime=False)
    assert [r.id for r in res] == [q.id for q in reqs]
    assert all(r.error is None for r in res)
    assert max(r.batch_size for r in res) > 1
    for q, r in zip(reqs, res):
        P = plans[q.matrix]
        if q.kind == "chebyshev":
            alone = P.run_recur(q.x, *mpk.chebyshev_coefficients(q.p))
        elif q.kind == "time_step":
            alone = P.cheb_time_step(q.x, q.dt, q.p)
        else:
            alone = P.run(q.x, q.p)
        torch.cuda.synchronize()
        assert r.Y.shape == alone.shape and torch.equal(r.Y, alone), (q.id, q.kind)
    st = serve.summarize(res, reqs, plans)
    assert sorted(st["by_matrix"]) == [0, 1, 2]
    assert sum(v["requests"] for v in st["by_matrix"].values()) == len(reqs)
    for m, v in st["by_matrix"].items():
        assert v["n"] == mats[m].n and v["p99_ms"] >= v["p50_ms"] > 0
        assert v["device_p99_ms"] >= v["device_p50_ms"] > 0 and v["queue_p99_ms"] >= 0
    with pytest.raises(ValueError):
        serve.Server(plans, use_baseline=[True])
    for P in plans:
        P.close()
