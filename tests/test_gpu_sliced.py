"""GPU: the sliced matrix layout (64-row slices stored slot by slot, one
thread per row and right-hand side) gives the same bits as the oracle and as
the LDS-staged CSR rows, for every schedule, right-hand-side counts that do
and do not divide the workgroup, FP32-stored values, empty rows and rows
longer than their neighbours."""
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


def ragged_stencil():
    """A 3D 27-point stencil (22^3) with every 97th row emptied and every
    211th row given five extra entries: uneven rows that still pad to less
    than a quarter more than the stored entries."""
    A = w.stencil_3d27(22)
    rows, cols, vals = [], [], []
    g = np.random.default_rng(9)
    for i in range(A.n):
        c = list(A.col[A.rowptr[i]:A.rowptr[i + 1]])
        v = list(A.val[A.rowptr[i]:A.rowptr[i + 1]])
        if i % 97 == 5:
            c, v = [], []
        elif i % 211 == 7:
            extra = g.integers(0, A.n, size=5)
            c += [int(e) for e in extra]
            v += list(g.standard_normal(5))
        rows.append(len(c))
        cols += c
        vals += v
    rp = np.zeros(A.n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(rows)
    return w.CSR(A.n, rp, np.array(cols, dtype=np.int32), np.array(vals), "ragged27")


def test_which_plans_get_the_sliced_layout():
    for A, want in ((w.stencil_3d27(16), 1), (w.anderson_3d(10), 1), (w.stencil_2d5(50), 1),
                    (ragged_stencil(), 1), (w.banded_random(1 << 14, half_width=300), 0)):
        P = mpk.Plan(A, reorder="none")
        info = P.info()
        assert info["sliced_layout"] == want, A.name
        if want:
            assert A.nnz <= info["sliced_entries"] <= 1.25 * A.nnz + 64
        P.close()


@pytest.mark.parametrize("sched", ["wave", "powers", "steps", "diag", "xcd"])
@pytest.mark.parametrize("R", [1, 2, 3, 5, 8, 16])
def test_sliced_rows_equal_oracle(sched, R):
    A = ragged_stencil()
    x = dev_x(A.n, R, 40 + R)
    ref = oracle.powers(A, x.cpu().numpy(), 5)
    for reorder in ("none", "bfs"):
        P = mpk.Plan(A, reorder=reorder)
        assert P.info()["sliced_layout"] == 1
        P.tune(schedule=sched, chunk_nnz=900, lag=3)
        Y = P.run(x, 5)
        B = P.run_baseline(x, 5)
        P.sync()
        assert torch.equal(Y, B), (sched, R, reorder)
        assert np.array_equal(Y.cpu().numpy(), ref), (sched, R, reorder)
        P.close()


@pytest.mark.parametrize("R", [1, 4, 7])
def test_sliced_rows_fp32_values_and_recurrence(R):
    A = w.anderson_3d(12)
    x = dev_x(A.n, R, 70 + R)
    coefs = mpk.chebyshev_coefficients(9)
    ref = oracle.recur(A, x.cpu().numpy(), *coefs, value_bits=32)
    P = mpk.Plan(A, value_bits=32, reorder="none")
    assert P.info()["sliced_layout"] == 1
    for sched in ("wave", "steps"):
        P.tune(schedule=sched, chunk_nnz=1000, lag=2)
        Y = P.run_recur(x, *coefs)
        B = P.run_baseline_recur(x, *coefs)
        P.sync()
        assert torch.equal(Y, B)
        assert np.array_equal(Y.cpu().numpy(), ref)
    P.close()


def test_sliced_rows_time_step_sums():
    A = w.anderson_3d(10)
    x = dev_x(A.n, 4, 91)
    al, be, ga, wa, wb = mpk.cheb_time_coefficients(10, 0.5)
    P = mpk.Plan(A, reorder="none")
    assert P.info()["sliced_layout"] == 1
    ra, rb = oracle.poly_sums(A, x.cpu().numpy(), al, be, ga, wa, wb)
    for baseline in (False, True):
        run = P.run_baseline_poly if baseline else P.run_poly
        acc, _ = run(x, wa, wb, al, be, ga)
        P.sync()
        got = acc.cpu().numpy()
        assert np.array_equal(got[0], ra) and np.array_equal(got[1], rb), baseline
    P.close()


def with_far_entries(A, far, every, seed):
    """A copy of A where every `every`-th row gets one more entry at column
    row + far (or row - far where that falls outside), value N(0,1)."""
    g = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(A.n):
        c = list(A.col[A.rowptr[i]:A.rowptr[i + 1]])
        v = list(A.val[A.rowptr[i]:A.rowptr[i + 1]])
        if i % every == 3:
            j = i + far if i + far < A.n else i - far
            if 0 <= j < A.n and j not in c:
                c.append(j)
                v.append(float(g.standard_normal()))
        rows.append(len(c))
        cols += c
        vals += v
    rp = np.zeros(A.n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(rows)
    return w.CSR(A.n, rp, np.array(cols, dtype=np.int32), np.array(vals), f"far{far}")


@pytest.mark.parametrize("far, bits", [(32767, 16), (32768, 32), (39000, 32)])
def test_column_offsets_16_and_32_bits(far, bits):
    """The sliced layout stores columns as 16-bit offsets from the row
    (modulo n, into [-n/2, n/2)) when every entry lies within 32767 of its
    row that way, else as columns; both give the oracle's bits.  A 42^3
    stencil (n = 74088) with a few entries exactly at the limit or beyond it
    (39000 is 35088 the other way round)."""
    A = with_far_entries(w.stencil_3d27(42), far, 499, far)
    assert max(abs(int(c) - i) for i in range(A.n)
               for c in A.col[A.rowptr[i]:A.rowptr[i + 1]]) == far
    for R in (1, 3):
        x = dev_x(A.n, R, 7 + R)
        ref = oracle.powers(A, x.cpu().numpy(), 4)
        P = mpk.Plan(A, reorder="none")
        info = P.info()
        assert info["sliced_layout"] == 1 and info["sliced_col_bits"] == bits
        for sched in ("wave", "powers", "steps"):
            P.tune(schedule=sched, chunk_nnz=4000, lag=4)
            Y = P.run(x, 4)
            B = P.run_baseline(x, 4)
            P.sync()
            assert torch.equal(Y, B), (far, R, sched)
            assert np.array_equal(Y.cpu().numpy(), ref), (far, R, sched)
        P.close()


def test_stencils_read_16_bit_offsets():
    for A in (w.stencil_3d27(16), w.stencil_2d5(50), ragged_stencil()):
        P = mpk.Plan(A, reorder="none")
        assert P.info()["sliced_col_bits"] == 16, A.name
        P.close()
    # a periodic lattice: the wrap-around neighbours lie n - 1600 away in
    # index, 1600 modulo n
    A = w.anderson_3d(40)
    assert max(abs(int(c) - i) for i in range(A.n)
               for c in A.col[A.rowptr[i]:A.rowptr[i + 1]]) > 32767
    x = dev_x(A.n, 2, 5)
    ref = oracle.powers(A, x.cpu().numpy(), 5)
    for vb in (64, 32):
        P = mpk.Plan(A, reorder="none", value_bits=vb)
        assert P.info()["sliced_col_bits"] == 16
        P.tune(schedule="wave", chunk_nnz=3000, lag=3)
        Y = P.run(x, 5)
        B = P.run_baseline(x, 5)
        P.sync()
        assert torch.equal(Y, B)
        if vb == 64:
            assert np.array_equal(Y.cpu().numpy(), ref)
        else:
            assert np.array_equal(Y.cpu().numpy(),
                                  oracle.powers(A, x.cpu().numpy(), 5, value_bits=32))
        P.close()
    P = mpk.Plan(w.banded_random(1 << 14, half_width=300), reorder="none")
    assert P.info()["sliced_col_bits"] == 0     # no sliced layout
    P.close()
