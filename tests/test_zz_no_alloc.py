"""GPU: mpk_run_noalloc (dependency workspace in the library's static device
array, nothing allocated) returns exactly what mpk_run returns, on two calls
in a row that share the array, the second with a smaller input."""
import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mpk = pytest.importorskip("paper_2405_12525_amd")


def dev_x(n, R, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.uniform(-1, 1, size=(n, R))).cuda()


def pinned_status():
    return torch.full((1,), 7, dtype=torch.int32).pin_memory()


def test_noalloc_equals_run_on_two_calls_the_second_smaller():
    torch.cuda.set_device(0)
    big, small = w.stencil_3d27(22), w.stencil_2d5(60)
    mpk.use_torch_allocator(True)   # every library device allocation is counted
    try:
        P1 = mpk.Plan(big, reorder="none")
        P1.tune(schedule="wave", chunk_nnz=1500, lag=3)
        P2 = mpk.Plan(small)
        P2.tune(schedule="powers", chunk_nnz=600)
        p1, R1, p2, R2 = 7, 3, 4, 1
        P1.prepare(p1, R1)
        P2.prepare(p2, R2)
        assert P1.schedule(p1)["n_chunks"] > P2.schedule(p2)["n_chunks"] > 1
        x1, x2 = dev_x(big.n, R1, 1), dev_x(small.n, R2, 2)
        Y1 = torch.empty((p1, big.n, R1), dtype=torch.float64, device="cuda")
        Y2 = torch.empty((p2, small.n, R2), dtype=torch.float64, device="cuda")
        s1, s2 = pinned_status(), pinned_status()
        torch.cuda.synchronize()
        allocs = mpk.allocator_stats["allocs"]
        P1.run_noalloc(x1, p1, Y1, status=s1)
        P2.run_noalloc(x2, p2, Y2, status=s2)   # reuses the array the first call left behind
        torch.cuda.synchronize()
        assert mpk.allocator_stats["allocs"] == allocs, "the no-allocation run allocated"
        assert int(s1[0]) == 0 and int(s2[0]) == 0
        ref1, ref2 = P1.run(x1, p1), P2.run(x2, p2)
        P1.sync()
        P2.sync()
        assert torch.equal(Y1, ref1) and torch.equal(Y2, ref2)
        assert np.array_equal(Y1.cpu().numpy(), oracle.powers(big, x1.cpu().numpy(), p1))
        assert np.array_equal(Y2.cpu().numpy(), oracle.powers(small, x2.cpu().numpy(), p2))
        P1.close()
        P2.close()
    finally:
        mpk.use_torch_allocator(False)


def test_noalloc_refuses_unprepared_and_oversized_schedules():
    torch.cuda.set_device(0)
    A = w.stencil_2d5(30)
    P = mpk.Plan(A)
    x = dev_x(A.n, 1, 3)
    Y = torch.empty((3, A.n, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(mpk.MPKError) as e:
        P.run_noalloc(x, 3, Y)
    assert e.value.status == mpk._capi.MPK_EINVAL and "prepare" in str(e.value)
    P.close()
    B = w.stencil_2d5(560)          # 313,600 one-row chunks: above the 1 MiB array
    Q = mpk.Plan(B, reorder="none")
    Q.tune(schedule="diag", chunk_nnz=1)
    Q.prepare(2, 1)
    xb = dev_x(B.n, 1, 4)
    Yb = torch.empty((2, B.n, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(mpk.MPKError) as e:
        Q.run_noalloc(xb, 2, Yb)
    assert e.value.status == mpk._capi.MPK_EUNSUPPORTED
    Q.close()
