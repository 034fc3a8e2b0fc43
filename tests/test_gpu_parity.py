"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every kernel forms each entry as the plain CSR sum (products rounded one by
one, added in stored order, no fused multiply-add), which is also what the
oracle computes, so the bar is bit-for-bit equality with the oracle for FP64
and for FP32-stored values (oracle on the same float-rounded values), and
level-blocked == baseline.  The tolerance bars of the specification are
checked as well: <= 1e-12 relative error per power for FP64 and <= 1e-5 for
FP32-stored values against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as w
from tests._util import rel_err_per_power

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mpk = pytest.importorskip("paper_2405_12525_amd")

TOL64, TOL32 = 1e-12, 1e-5


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


def run_both(P, x, p, recur=None):
    xd = dev(x)
    if recur is None:
        Y = P.run(xd, p)
        B = P.run_baseline(xd, p)
    else:
        Y = P.run_recur(xd, *recur)
        B = P.run_baseline_recur(xd, *recur)
    P.sync()
    return host(Y), host(B)


# ------------------------------------------------------------------ small configurations

SCHEDS = ["steps", "wave", "diag", "powers", "xcd"]


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("reorder,order", [("bfs", "original"), ("none", "original"),
                                           ("bfs", "plan")])
def test_stencil2d_p4_matches_oracle(sched, reorder, order):
    A, x, p, _ = w.config("stencil2d5_64_p4")
    P = mpk.Plan(A, reorder=reorder, order=order)
    P.tune(schedule=sched, chunk_nnz=512)
    if order == "plan":
        lp, perm = P.levels()
        Ap = oracle.permute_csr(A, perm)
        xp = x[perm]
        ref = oracle.powers(Ap, xp, p)
        Y, B = run_both(P, xp, p)
    else:
        ref = oracle.powers(A, x, p)
        Y, B = run_both(P, x, p)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, ref)
    assert rel_err_per_power(Y, ref).max() <= TOL64


@pytest.mark.parametrize("chunk_nnz,workgroups", [(64, 0), (1000, 7), (20000, 0), (3000, 300)])
def test_integer_inputs_bit_exact(chunk_nnz, workgroups):
    A = w.stencil_3d27(20)
    x = w.integer_vectors(A.n, 1, 42)
    P = mpk.Plan(A)
    P.tune(chunk_nnz=chunk_nnz, workgroups=workgroups)
    Y, B = run_both(P, x, 6)
    assert np.array_equal(Y, oracle.powers(A, x, 6))
    assert np.array_equal(B, Y)


def ragged_matrix(n, seed):
    """Irregular rows (empty, short, long, one dense-ish) with a non-symmetric pattern."""
    g = w.rng(seed)
    lens = g.integers(0, 30, size=n)
    lens[g.integers(0, n, size=n // 20)] = 0
    lens[n // 3] = min(n, 900)
    rows, cols = [], []
    for i in range(n):
        c = np.unique(np.clip(i + g.integers(-200, 201, size=lens[i]), 0, n - 1))
        rows.append(np.full(c.size, i))
        cols.append(c)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    vals = g.standard_normal(cols.size) * 0.2
    return w.CSR(n, rowptr, cols.astype(np.int32), vals, f"ragged_{n}")


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5, 7, 8, 12, 16])
def test_ragged_multi_rhs(R):
    A = ragged_matrix(5003, 7)
    x = w.uniform_vectors(A.n, R, 100 + R)
    p = 5
    ref = oracle.powers(A, x, p)
    P = mpk.Plan(A)
    P.tune(chunk_nnz=700)
    Y, B = run_both(P, x, p)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, ref)
    # every column equals its own single right-hand-side run
    for r in range(R):
        Y1, _ = run_both(P, x[:, r:r + 1], p)
        assert np.array_equal(Y[:, :, r:r + 1], Y1)


@pytest.mark.parametrize("tune", [dict(schedule="wave"), dict(schedule="diag"),
                                  dict(schedule="powers"), dict(schedule="xcd"),
                                  dict(schedule="xcd", workgroups=5),
                                  dict(schedule="xcd", chunk_nnz=50, workgroups=64),
                                  dict(schedule="wave", seg_powers=1), dict(seg_powers=3),
                                  dict(schedule="xcd", seg_powers=2),
                                  dict(schedule="wave", skip_ahead=4, lag=3),
                                  dict(schedule="powers", skip_ahead=1),
                                  dict(schedule="diag", skip_ahead=8, chunk_nnz=300),
                                  dict(lag=1), dict(lag=5000), dict(chunk_nnz=50, workgroups=3),
                                  dict(cache_bytes=1 << 16)])
def test_tuning_never_changes_a_bit(tune):
    A = w.anderson_3d(12)
    x = w.uniform_vectors(A.n, 8, 5)
    P = mpk.Plan(A)
    Y0, _ = run_both(P, x, 4)
    P.tune(**tune)
    Y1, B1 = run_both(P, x, 4)
    assert np.array_equal(Y0, Y1) and np.array_equal(Y1, B1)
    assert np.array_equal(Y1, oracle.powers(A, x, 4))


def test_fp32_values():
    A = w.banded_random(60000, half_width=500, window=4096)
    x = w.uniform_vectors(A.n, 1, 1003)
    p = 6
    P = mpk.Plan(A, value_bits=32)
    P.tune(chunk_nnz=4096)
    Y, B = run_both(P, x, p)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, oracle.powers(A, x, p, value_bits=32))
    assert rel_err_per_power(Y, oracle.powers(A, x, p)).max() <= TOL32


@pytest.mark.parametrize("value_bits", [64, 32])
def test_chebyshev_recurrence(value_bits):
    A = w.anderson_3d(24)
    x = w.random_sign_unit_vectors(A.n, 8, 1004)
    p = 16
    coefs = oracle.chebyshev_coefficients(p)
    P = mpk.Plan(A, value_bits=value_bits)
    P.tune(chunk_nnz=2000)
    Y, B = run_both(P, x, p, recur=coefs)
    assert np.array_equal(Y, B)
    tol = TOL64 if value_bits == 64 else TOL32
    assert np.array_equal(Y, oracle.recur(A, x, *coefs, value_bits=value_bits))
    assert rel_err_per_power(Y, oracle.recur(A, x, *coefs)).max() <= tol


def test_general_recurrence_coefficients():
    A = ragged_matrix(3001, 3)
    x = w.uniform_vectors(A.n, 2, 9)
    g = w.rng(77)
    a, b, c = g.uniform(-1, 1, 9), g.uniform(-1, 1, 9), g.uniform(-1, 1, 9)
    P = mpk.Plan(A)
    P.tune(chunk_nnz=500)
    Y, B = run_both(P, x, 9, recur=(a, b, c))
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, oracle.recur(A, x, a, b, c))


def test_long_p_spans_segments():
    A = w.anderson_3d(10)
    x = w.uniform_vectors(A.n, 2, 3)
    p = 150  # three kernel launches of at most 64 powers
    P = mpk.Plan(A)
    Y, B = run_both(P, x, p)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, oracle.powers(A, x, p))
    coefs = oracle.chebyshev_coefficients(p)
    Yc, Bc = run_both(P, x, p, recur=coefs)
    assert np.array_equal(Yc, Bc)
    assert np.array_equal(Yc, oracle.recur(A, x, *coefs))


def test_split_invariant_and_plan_order_permutation():
    A = w.stencil_2d5(50)
    x = w.uniform_vectors(A.n, 2, 8)
    P = mpk.Plan(A)
    Y, _ = run_both(P, x, 7)
    Ya, _ = run_both(P, x, 3)
    Yb, _ = run_both(P, Ya[-1], 4)
    assert np.array_equal(Y, np.concatenate([Ya, Yb]))
    # PLAN order: permute in, run, permute out == ORIGINAL order, bit for bit
    Q = mpk.Plan(A, order="plan")
    xp = Q.permute(dev(x), to_plan=True)
    Yp = Q.run(xp, 7)
    Yo = Q.permute(Yp, to_plan=False)
    assert np.array_equal(host(Yo), Y)


def test_edge_cases():
    # empty matrix
    E = w.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    P = mpk.Plan(E)
    Y = P.run(torch.zeros((0, 1), dtype=torch.float64, device="cuda"), 3)
    assert Y.shape == (3, 0, 1)
    # one row
    one = w.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([0.5]))
    Y, B = run_both(mpk.Plan(one), np.array([[2.0]]), 4)
    assert Y[:, 0, 0].tolist() == [1.0, 0.5, 0.25, 0.125]
    # all-empty rows
    Z = w.CSR(5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0))
    Y, B = run_both(mpk.Plan(Z), np.ones((5, 1)), 2)
    assert np.array_equal(Y, np.zeros((2, 5, 1)))
    # disconnected graph + a dense row
    A = w.random_sparse(700, 0.002, 11)
    D = A.to_dense()
    D[350, :] = 0.01
    A = w.from_dense(D)
    x = w.uniform_vectors(A.n, 1, 2)
    P = mpk.Plan(A)
    P.tune(chunk_nnz=64)
    Y, B = run_both(P, x, 5)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, oracle.powers(A, x, 5))


def test_identity_and_permutation_exact():
    A = w.identity(3000)
    x = w.uniform_vectors(3000, 4, 1)
    Y, _ = run_both(mpk.Plan(A), x, 3)
    assert all(np.array_equal(Y[k], x) for k in range(3))
    Pm, sigma = w.permutation_matrix(4000, 5)
    x = w.uniform_vectors(4000, 1, 2)
    Y, _ = run_both(mpk.Plan(Pm), x, 4)
    idx = np.arange(4000)
    for k in range(4):
        idx = sigma[idx]
        assert np.array_equal(Y[k], x[idx])


@pytest.mark.parametrize("sched,skip", [("wave", 0), ("xcd", 0), ("wave", 3)])
def test_wait_limit_reports_timeout_and_recovers(sched, skip):
    A = w.stencil_3d27(40)
    x = w.uniform_vectors(A.n, 1, 4)
    P = mpk.Plan(A)
    P.tune(schedule=sched, spin_limit_us=1, chunk_nnz=2000, skip_ahead=skip, lag=1)
    seen_timeout = False
    for _ in range(3):
        P.run(dev(x), 24)
        try:
            P.sync()
        except mpk.MPKError as e:
            assert "MPK_ETIMEOUT" in str(e)
            seen_timeout = True
    assert seen_timeout
    P.tune(spin_limit_us=0, chunk_nnz=2000, lag=0)
    Y, B = run_both(P, x, 6)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, oracle.powers(A, x, 6))


@pytest.mark.parametrize("sched,skip", [("steps", 0), ("wave", 0), ("xcd", 0), ("wave", 4)])
def test_concurrent_streams_share_a_plan(sched, skip):
    A = w.stencil_3d27(24)
    xs = [w.uniform_vectors(A.n, 2, s) for s in range(4)]
    P = mpk.Plan(A)
    P.tune(schedule=sched, chunk_nnz=1500, skip_ahead=skip)
    streams = [torch.cuda.Stream() for _ in xs]
    outs = []
    xds = [dev(x) for x in xs]
    torch.cuda.synchronize()
    for xd, s in zip(xds, streams):
        with torch.cuda.stream(s):
            outs.append(P.run(xd, 5, stream=s))
    P.sync()
    for x, Y in zip(xs, outs):
        assert np.array_equal(host(Y), oracle.powers(A, x, 5))


@pytest.mark.parametrize("seg", [1, 2, 5])
def test_segmented_recurrence_matches_oracle(seg):
    A = w.anderson_3d(11)
    x = w.random_sign_unit_vectors(A.n, 2, 9)
    P = mpk.Plan(A, value_bits=32)
    P.tune(schedule="wave", seg_powers=seg, chunk_nnz=700)
    coefs = mpk.chebyshev_coefficients(7)
    Y, B = run_both(P, x, 7, recur=coefs)
    ref = oracle.recur(A, x, *coefs, value_bits=32)
    assert np.array_equal(Y, ref) and np.array_equal(B, ref)


@pytest.mark.parametrize("sched", ["wave", "xcd", "powers", "steps"])
@pytest.mark.parametrize("R", [4, 6, 16])
def test_multi_rhs_schedules_fp32(sched, R):
    A = w.anderson_3d(14)
    x = w.random_sign_unit_vectors(A.n, R, 40 + R)
    P = mpk.Plan(A, value_bits=32)
    P.tune(schedule=sched, chunk_nnz=900)
    coefs = mpk.chebyshev_coefficients(6)
    Y, B = run_both(P, x, 6, recur=coefs)
    ref = oracle.recur(A, x, *coefs, value_bits=32)
    assert np.array_equal(Y, ref) and np.array_equal(B, ref)
    ref64 = oracle.recur(A, x, *coefs)
    assert rel_err_per_power(Y, ref64).max() <= TOL32


def test_zero_coefficient_omits_its_term():
    A = w.CSR(2, np.array([0, 0, 1], np.int32), np.array([1], np.int32), np.array([2.0]), "t")
    x = np.array([[np.inf], [1.0]])
    P = mpk.Plan(A)
    for beta in (0.0, 1.0):
        coefs = (np.array([3.0, 2.0]), np.array([beta, 0.0]), np.array([0.0, -1.0]))
        ref = oracle.recur(A, x, *coefs)
        Y, B = run_both(P, x, 2, recur=coefs)
        assert np.array_equal(Y, ref, equal_nan=True) and np.array_equal(B, ref, equal_nan=True)


# ------------------------------------------------------------------ full-size workloads

@pytest.mark.slow
def test_full_stencil3d27_128_p8():
    A, x, p, _ = w.config("stencil3d27_128_p8")
    P = mpk.Plan(A)
    xi = w.integer_vectors(A.n, 1, 1002)
    Yi, Bi = run_both(P, xi, p)
    assert np.array_equal(Yi, oracle.powers(A, xi, p))
    assert np.array_equal(Yi, Bi)
    Y, B = run_both(P, x, p)
    assert np.array_equal(Y, B)
    ref = oracle.powers(A, x, p)
    assert np.array_equal(Y, ref)
    assert rel_err_per_power(Y, ref).max() <= TOL64


@pytest.mark.slow
def test_full_anderson160_chebyshev16_r8_fp32():
    A, x, p, _ = w.config("anderson160_cheb16_r8")
    coefs = oracle.chebyshev_coefficients(p)
    P = mpk.Plan(A, value_bits=32)
    Y, B = run_both(P, x, p, recur=coefs)
    assert np.array_equal(Y, B)
    assert np.array_equal(Y, oracle.recur(A, x, *coefs, value_bits=32))
    assert rel_err_per_power(Y, oracle.recur(A, x, *coefs)).max() <= TOL32


# the launch configuration the benchmark times: the workloads' own order and
# the autotuner's choice (whichever it picks, the result is the oracle's)

@pytest.mark.slow
@pytest.mark.parametrize("name,vb", [("stencil3d27_128_p8", 64), ("banded_4m_p6", 64),
                                     ("banded_4m_p6", 32), ("stencil3d27_64_p16_r16", 64),
                                     ("anderson160_cheb16_r8", 32)])
def test_full_size_autotuned_original_order(name, vb):
    A, x, p, kind = w.config(name)
    cheb = kind == "chebyshev"
    coefs = oracle.chebyshev_coefficients(p) if cheb else None
    xd = dev(x)
    P = mpk.Plan(A, reorder="none", value_bits=vb)
    P.autotune(xd, p, reps=1, recur=cheb, force=True)
    Y, B = run_both(P, x, p, recur=coefs)
    ref = (oracle.recur(A, x, *coefs, value_bits=vb) if cheb
           else oracle.powers(A, x, p, value_bits=vb))
    assert np.array_equal(Y, ref) and np.array_equal(B, ref)
    P.close()


# ------------------------------------------------------------------ device-built plans

def _host_levels(A, **kw):
    return mpk.Plan(A, device=mpk.MPK_DEVICE_NONE, **kw).levels()


def _with_dense_rows(n, seed):
    """A sparse random pattern where rows 0, 7 and n/2 (and their columns)
    are dense: frontier vertices with hundreds of neighbours, which the
    device BFS checks 64 at a time over several rounds."""
    g = np.random.default_rng(seed)
    m = g.random((n, n)) < 0.001
    for r in (0, 7, n // 2):
        m[r, g.random(n) < 0.3] = True
    m = m | m.T
    np.fill_diagonal(m, True)
    return w.from_dense(np.where(m, g.standard_normal((n, n)), 0.0), "dense_rows")


@pytest.mark.parametrize("case", ["stencil", "random_sym", "random_nonsym", "disconnected",
                                  "empty_rows", "anderson", "dense_rows"])
@pytest.mark.parametrize("order", ["original", "plan"])
def test_device_levels_equal_host_levels(case, order):
    # BFS levels and the permutation computed on the GPU are the host
    # planner's exactly (integers), and runs on the device-built plan match
    # the oracle bit for bit
    A = {"stencil": lambda: w.stencil_3d27(16),
         "random_sym": lambda: w.random_sparse(3000, 0.002, 41, symmetric_pattern=True),
         "random_nonsym": lambda: w.random_sparse(3000, 0.0015, 42),
         "disconnected": lambda: w.random_sparse(2500, 0.0004, 43, symmetric_pattern=True),
         "empty_rows": lambda: w.CSR(6, np.array([0, 0, 2, 2, 3, 3, 3], np.int32),
                                     np.array([4, 1, 2], np.int32), np.array([1.0, 2.0, 3.0])),
         "anderson": lambda: w.anderson_3d(12),
         "dense_rows": lambda: _with_dense_rows(3000, 45)}[case]()
    for root in (0, A.n // 2):
        P = mpk.Plan(A, order=order, root=root)
        lp, perm = P.levels()
        lh, permh = _host_levels(A, order=order, root=root)
        assert np.array_equal(lp, lh) and np.array_equal(perm, permh), (case, root)
        x = w.uniform_vectors(A.n, 2, 7)
        if order == "plan":
            Ap = oracle.permute_csr(A, perm)
            Y, B = run_both(P, x[perm], 4)
            ref = oracle.powers(Ap, x[perm], 4)
        else:
            Y, B = run_both(P, x, 4)
            ref = oracle.powers(A, x, 4)
        assert np.array_equal(Y, ref) and np.array_equal(B, ref)
        P.close()


def test_device_levels_fp32_and_many_components():
    # FP32 values are converted by the device permutation; a graph with more
    # components than the device search takes goes through the host planner
    A = w.anderson_3d(10)
    P = mpk.Plan(A, value_bits=32)
    x = w.uniform_vectors(A.n, 1, 8)
    Y, B = run_both(P, x, 3)
    assert np.array_equal(Y, oracle.powers(A, x, 3, value_bits=32))
    n = 500   # a diagonal matrix: 500 components
    D = w.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
              np.linspace(0.5, 1.5, n))
    Q = mpk.Plan(D)
    lp, perm = Q.levels()
    assert len(lp) - 1 == n and np.array_equal(perm, np.arange(n))
    Y, B = run_both(Q, np.ones((n, 1)), 2)
    assert np.array_equal(Y, oracle.powers(D, np.ones((n, 1)), 2))
    P.close()
    Q.close()


def _device_csr(A):
    import types
    return types.SimpleNamespace(
        n=A.n, rowptr=torch.from_numpy(np.ascontiguousarray(A.rowptr, np.int32)).cuda(),
        col=torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).cuda(),
        val=torch.from_numpy(np.ascontiguousarray(A.val, np.float64)).cuda())


@pytest.mark.parametrize("reorder,order,vb", [("bfs", "original", 64), ("none", "original", 64),
                                              ("bfs", "plan", 32), ("none", "plan", 32)])
@pytest.mark.parametrize("case", ["stencil", "random_nonsym", "disconnected"])
def test_plan_from_device_csr_equals_host_plan(reorder, order, vb, case):
    A = {"stencil": lambda: w.stencil_3d27(14),
         "random_nonsym": lambda: w.random_sparse(2000, 0.002, 44),
         "disconnected": lambda: w.random_sparse(1500, 0.0005, 45, symmetric_pattern=True)}[case]()
    P = mpk.Plan(_device_csr(A), reorder=reorder, order=order, value_bits=vb)
    Q = mpk.Plan(A, reorder=reorder, order=order, value_bits=vb)
    lp, perm = P.levels()
    lq, permq = Q.levels()
    assert np.array_equal(lp, lq) and np.array_equal(perm, permq)
    ip, iq = P.info(), Q.info()
    same = ("n", "nnz", "n_levels", "max_level_rows", "matrix_bytes", "fingerprint",
            "sliced_layout", "sliced_col_bits")
    assert {k: ip[k] for k in same} == {k: iq[k] for k in same}
    x = w.uniform_vectors(A.n, 2, 9)
    xs = x[perm] if order == "plan" else x
    Y, B = run_both(P, xs, 4)
    Yq, _ = run_both(Q, xs, 4)
    assert np.array_equal(Y, Yq) and np.array_equal(B, Yq)
    P.tune(schedule="xcd", chunk_nnz=800)   # exact dependency lists: columns read back
    Yx, _ = run_both(P, xs, 4)
    assert np.array_equal(Yx, Yq)
    P.close()
    Q.close()


def test_plan_from_device_csr_checks_and_fallbacks():
    A = w.stencil_2d5(12)
    D = _device_csr(A)
    bad = _device_csr(A)
    bad.col[5] = A.n                      # a column out of range
    with pytest.raises(mpk.MPKError):
        mpk.Plan(bad)
    bad = _device_csr(A)
    bad.rowptr[3] = bad.rowptr[2] - 1     # a row pointer that decreases
    with pytest.raises(mpk.MPKError):
        mpk.Plan(bad)
    # the pseudo-peripheral root and a 400-component graph go through the host
    P = mpk.Plan(D, root="peripheral")
    Q = mpk.Plan(A, root="peripheral")
    assert np.array_equal(P.levels()[1], Q.levels()[1])
    n = 400
    Dg = w.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.linspace(0.5, 1.5, n))
    R = mpk.Plan(_device_csr(Dg))
    assert len(R.levels()[0]) - 1 == n
    Y, B = run_both(R, np.ones((n, 1)), 2)
    assert np.array_equal(Y, oracle.powers(Dg, np.ones((n, 1)), 2))
    # the autotuner's cache key is the same for both constructions
    xd = dev(w.uniform_vectors(A.n, 1, 3))
    t = Q.autotune(xd, 4, reps=1, force=True)
    import time
    t0 = time.perf_counter()
    t2 = mpk.Plan(D, root="peripheral").autotune(xd, 4)
    assert time.perf_counter() - t0 < 0.5 and t2["schedule"] == t["schedule"]
    for X in (P, Q, R):
        X.close()
