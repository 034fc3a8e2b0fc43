"""GPU: plans in sub-level order (BFS levels, each ordered by the distance
from a second root) give the oracle's bits for every schedule, both task
orders, several right-hand-side counts, the recurrence and FP32 values; the
same plan from a device CSR equals the host one; and plans rooted at a
pseudo-peripheral row, from a host and from a device CSR, carry the oracle's
levels and results."""
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


def device_csr(A):
    import types
    return types.SimpleNamespace(n=A.n, rowptr=torch.from_numpy(A.rowptr).cuda(),
                                 col=torch.from_numpy(A.col).cuda(),
                                 val=torch.from_numpy(A.val).cuda())


MATS = {"cube": lambda: w.stencil_3d27(19), "anderson": lambda: w.anderson_3d(13),
        "rand": lambda: w.random_sparse(3000, 0.002, 11, symmetric_pattern=False)}


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("sched", ["steps", "wave", "diag", "powers", "xcd"])
def test_sublevel_plans_equal_oracle(name, sched):
    A = MATS[name]()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    P = mpk.Plan(A, reorder="sublevels")
    lp, perm = P.levels()
    assert np.array_equal(perm, oracle.sublevels(A.n, A.rowptr, A.col, 0)[2])
    for R, dyn in ((1, 0), (3, 1), (8, 0)):
        P.tune(schedule=sched, chunk_nnz=1200, workgroups=2 * cus, dynamic_tickets=dyn)
        x = dev_x(A.n, R, 100 + R)
        Y = P.run(x, 6)
        B = P.run_baseline(x, 6)
        torch.cuda.synchronize()
        P.sync()
        ref = oracle.powers(A, x.cpu().numpy(), 6)
        assert np.array_equal(Y.cpu().numpy(), ref), (sched, R)
        assert torch.equal(Y, B)
    P.close()


def test_sublevel_plans_recurrence_and_fp32_values():
    A = w.anderson_3d(14)
    P = mpk.Plan(A, reorder="sublevels", value_bits=32)
    P.tune(schedule="xcd", chunk_nnz=900)
    x = dev_x(A.n, 4, 7)
    coefs = mpk.chebyshev_coefficients(9)
    Y = P.run_recur(x, *coefs)
    torch.cuda.synchronize()
    P.sync()
    ref = oracle.recur(A, x.cpu().numpy(), *coefs, value_bits=32)
    assert np.array_equal(Y.cpu().numpy(), ref)
    P.close()


def test_sublevel_plan_from_device_csr_equals_host_plan():
    A = w.stencil_3d27(16)
    H = mpk.Plan(A, reorder="sublevels")
    D = mpk.Plan(device_csr(A), reorder="sublevels")
    assert np.array_equal(H.levels()[1], D.levels()[1])
    assert H.info()["sublevel_root"] == D.info()["sublevel_root"]
    x = dev_x(A.n, 2, 3)
    assert torch.equal(H.run(x, 5), D.run(x, 5))
    torch.cuda.synchronize()
    H.close()
    D.close()


@pytest.mark.parametrize("source", ["host", "device"])
@pytest.mark.parametrize("name", ["grid", "rand"])
def test_peripheral_root_plans(source, name):
    A = w.stencil_2d5(37) if name == "grid" else w.random_sparse(2500, 0.002, 21)
    src = A if source == "host" else device_csr(A)
    P = mpk.Plan(src, root="peripheral")
    r = oracle.pseudo_peripheral_root(A.n, A.rowptr, A.col)
    levels, operm, _ = oracle.bfs_levels(A.n, A.rowptr, A.col, root=r)
    lp, perm = P.levels()
    assert np.array_equal(perm, operm)
    assert [int(v) for v in lp] == [0] + np.cumsum([len(L) for L in levels]).tolist()
    for sched in ("wave", "powers"):
        P.tune(schedule=sched, chunk_nnz=1000)
        x = dev_x(A.n, 2, 40)
        Y = P.run(x, 5)
        torch.cuda.synchronize()
        P.sync()
        assert np.array_equal(Y.cpu().numpy(), oracle.powers(A, x.cpu().numpy(), 5)), sched
    P.close()
