"""GPU parity of the weighted power sums (one Chebyshev time step).

The kernels run the recurrence with a ring of two vectors and update the
sums in each power's epilogue; the oracle forms y_1..y_p in full and sums
them in increasing k with the same skipping of zero weights.  Products and
sums are rounded one by one in both, so the bar is bit-for-bit equality
(FP64 and FP32-stored values alike), level-blocked == p x SpMV, and the
ring's last two slots equal the oracle's y_{p-1} and y_p.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def weights(p, seed, zero_frac=0.3, lead=0):
    g = np.random.default_rng(seed)
    wv = g.uniform(-1.0, 1.0, p + 1)
    wv[g.random(p + 1) < zero_frac] = 0.0
    wv[:lead] = 0.0
    return wv


def check_poly(P, A, x, wa, wb, coefs, vb, baseline_too=True):
    p = wa.size - 1
    xd = dev(x)
    kw = {} if coefs is None else dict(zip(("alpha", "beta", "gamma"), coefs))
    acc, work = P.run_poly(xd, wa, wb, **kw)
    P.sync()
    ra, rb = oracle.poly_sums(A, x, *(coefs if coefs is not None else
                                      (np.ones(p), np.zeros(p), np.zeros(p))),
                              wa, wb, value_bits=vb)
    got = host(acc)
    assert np.array_equal(got[0], ra)
    if wb is not None:
        assert np.array_equal(got[1], rb)
    # the ring keeps y_{p-1} and y_p in slots (k-1) mod 2
    Y = oracle.recur(A, x, *(coefs if coefs is not None else
                             (np.ones(p), np.zeros(p), np.zeros(p))), value_bits=vb)
    ring = host(work)
    assert np.array_equal(ring[(p - 1) % 2], Y[p - 1])
    if p >= 2:
        assert np.array_equal(ring[(p - 2) % 2], Y[p - 2])
    if baseline_too:
        bacc, bwork = P.run_baseline_poly(xd, wa, wb, **kw)
        P.sync()
        assert np.array_equal(host(bacc), got)
        assert np.array_equal(host(bwork)[(p - 1) % 2], ring[(p - 1) % 2])


SCHEDS = ["steps", "wave", "diag", "powers", "xcd"]


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("R", [1, 2, 4, 8])
def test_chebyshev_sums_all_schedules(sched, R):
    A = w.stencil_3d27(18)
    x = w.uniform_vectors(A.n, R, 40 + R)
    p = 9
    P = mpk.Plan(A)
    P.tune(schedule=sched, chunk_nnz=3000)
    coefs = oracle.chebyshev_coefficients(p)
    check_poly(P, A, x, weights(p, 1), weights(p, 2, lead=3), coefs, 64)
    P.close()


@pytest.mark.parametrize("p", [1, 2, 3, 70])
def test_plain_powers_sums_edges(p):
    # p = 70 spans two segments of the persistent kernel (at most 64 powers
    # per launch), so the ring continues across a launch boundary
    A = w.stencil_2d5(40)
    x = w.uniform_vectors(A.n, 2, 7)
    # keep the values bounded: 1/8 of the 5-point Laplacian's norm bound
    A8 = w.CSR(A.n, A.rowptr, A.col, A.val / 8.0, "scaled")
    P8 = mpk.Plan(A8)
    P8.tune(schedule="wave", chunk_nnz=400)
    check_poly(P8, A8, x, weights(p, 3), weights(p, 4, zero_frac=0.0), None, 64)
    P8.close()


def test_segmented_run_and_zero_weight_patterns():
    A = w.anderson_3d(12)
    x = w.random_sign_unit_vectors(A.n, 4, 9)
    p = 12
    P = mpk.Plan(A)
    P.tune(schedule="powers", chunk_nnz=1500, seg_powers=5)
    coefs = oracle.chebyshev_coefficients(p)
    z = np.zeros(p + 1)
    only0 = z.copy(); only0[0] = 0.75
    lastonly = z.copy(); lastonly[p] = -2.0
    for wa, wb in ((z, None), (only0, lastonly), (weights(p, 5), z),
                   (weights(p, 6, lead=1), weights(p, 7))):
        check_poly(P, A, x, wa, wb, coefs, 64)
    P.close()


def test_fp32_values_anderson_time_step_matches_oracle():
    A = w.anderson_3d(20)
    g = np.random.default_rng(12)
    psi = g.standard_normal((A.n, 8))   # 4 complex states as column pairs
    P = mpk.Plan(A, value_bits=32)
    P.tune(schedule="wave", chunk_nnz=4000)
    M, dt = 16, 1.3
    al, be, ga, wa, wb = mpk.cheb_time_coefficients(M, dt)
    check_poly(P, A, psi, wa, wb, (al, be, ga), 32)
    out = host(P.cheb_time_step(dev(psi), dt, M))
    ra, rb = oracle.poly_sums(A, psi, al, be, ga, wa, wb, value_bits=32)
    assert np.array_equal(out, oracle.combine_complex(ra, rb))
    base = host(P.cheb_time_step(dev(psi), dt, M, baseline=True))
    assert np.array_equal(base, out)
    # against the oracle's own step (its Bessel weights from scipy): the
    # weights differ in the last bits only
    ref = oracle.cheb_time_step(A, psi, dt, M, value_bits=32)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    P.close()


def test_time_step_is_unitary_and_reversible_fp64():
    A = w.anderson_3d(16)
    g = np.random.default_rng(13)
    psi = g.standard_normal((A.n, 2))
    P = mpk.Plan(A)
    P.tune(schedule="xcd", chunk_nnz=2000)
    M, dt = 40, 4.0
    fwd = P.cheb_time_step(dev(psi), dt, M)
    back = host(P.cheb_time_step(fwd, -dt, M))
    f = host(fwd)
    # exp(-i dt H) is unitary and exp(+i dt H) undoes it; truncation after
    # M = 40 at dt = 4 leaves ~1e-30
    assert abs(np.linalg.norm(f) - np.linalg.norm(psi)) <= 1e-12 * np.linalg.norm(psi)
    assert np.abs(back - psi).max() <= 1e-12
    P.close()


def test_nonsymmetric_pattern_rejected_by_level_blocked_form():
    A = w.random_sparse(900, 0.004, 21)
    x = w.uniform_vectors(A.n, 1, 3)
    P = mpk.Plan(A)
    p = 6
    wa = weights(p, 8)
    with pytest.raises(mpk.MPKError):
        P.run_poly(dev(x), wa)
    acc, work = P.run_baseline_poly(dev(x), wa)
    P.sync()
    ra, _ = oracle.poly_sums(A, x, np.ones(p), np.zeros(p), np.zeros(p), wa)
    assert np.array_equal(host(acc)[0], ra)
    P.close()


def test_argument_checks():
    import ctypes
    A = w.stencil_2d5(12)
    P = mpk.Plan(A)
    x = dev(w.uniform_vectors(A.n, 2, 1))
    with pytest.raises(ValueError):
        P.run_poly(x, np.ones(1))                        # p = 0
    # sums placed inside the ring: rejected before any launch
    work = torch.empty((2, A.n, 2), dtype=torch.float64, device="cuda")
    wa = np.ones(4)
    rc = P._lib.mpk_run_poly(P._h, ctypes.c_void_p(x.data_ptr()), 3, 2, None, None, None,
                             wa.ctypes.data, None, ctypes.c_void_p(work.data_ptr()),
                             ctypes.c_void_p(work.data_ptr()), None)
    assert rc == mpk._capi.MPK_EINVAL
    with pytest.raises(mpk.MPKError):
        P.cheb_time_step(x, 1.0, 0)                      # M = 0
    with pytest.raises(ValueError):
        P.cheb_time_step(dev(w.uniform_vectors(A.n, 3, 2)), 1.0, 8)   # odd column count
    P.close()


@pytest.mark.parametrize("seg", [0, 1, 2, 3])
def test_flush_patterns_across_segments(seg):
    # each sum is flushed at most every third power and takes y_{m-2} and
    # y_{m-1} from the task at power m; segments of 1-3 powers put those
    # terms in the previous launch's outputs
    A = w.stencil_2d5(20)
    A = w.CSR(A.n, A.rowptr, A.col, A.val / 8.0, "scaled")
    P = mpk.Plan(A)
    P.tune(schedule="wave", chunk_nnz=300, seg_powers=seg)
    g = np.random.default_rng(500 + seg)
    for case in range(12):
        p = int(g.integers(1, 8))
        R = int(g.choice([1, 2, 4]))
        x = w.uniform_vectors(A.n, R, 600 + case)
        wa = g.uniform(-1, 1, p + 1) * (g.random(p + 1) < g.uniform(0.2, 0.9))
        wb = g.uniform(-1, 1, p + 1) * (g.random(p + 1) < g.uniform(0.2, 0.9))
        coefs = oracle.chebyshev_coefficients(p) if case % 2 else None
        check_poly(P, A, x, wa, wb, coefs, 64)
    P.close()


@pytest.mark.parametrize("R", [3, 5, 16])
def test_sums_generic_rhs_counts(R):
    # R = 3 and 5 run the generic instantiation; 16 the widest specialised one
    A = w.anderson_3d(10)
    x = w.uniform_vectors(A.n, R, 80 + R)
    P = mpk.Plan(A, value_bits=32)
    P.tune(schedule="wave", chunk_nnz=900)
    p = 7
    check_poly(P, A, x, weights(p, 90 + R), weights(p, 91 + R), oracle.chebyshev_coefficients(p), 32)
    P.close()


def test_sums_in_plan_order():
    # vectors in the BFS numbering: the same sums as the oracle on P A P^T
    A = w.stencil_3d27(14)
    P = mpk.Plan(A, order="plan")
    _, perm = P.levels()
    Ap = oracle.permute_csr(A, perm)
    x = w.uniform_vectors(A.n, 2, 95)
    p = 6
    check_poly(P, Ap, x, weights(p, 96), weights(p, 97), oracle.chebyshev_coefficients(p), 64)
    P.close()


def test_sums_on_concurrent_streams():
    # runs on one plan from several streams draw separate dependency
    # workspaces; each call has its own ring and sums
    A = w.stencil_3d27(20)
    P = mpk.Plan(A)
    P.tune(schedule="wave", chunk_nnz=1500)
    p = 8
    coefs = oracle.chebyshev_coefficients(p)
    xs = [w.uniform_vectors(A.n, 2, 120 + i) for i in range(3)]
    ws = [(weights(p, 130 + i), weights(p, 140 + i)) for i in range(3)]
    streams = [torch.cuda.Stream() for _ in xs]
    xds = [dev(x) for x in xs]
    torch.cuda.synchronize()
    outs = []
    for xd, (wa, wb), s in zip(xds, ws, streams):
        with torch.cuda.stream(s):
            outs.append(P.run_poly(xd, wa, wb, *coefs, stream=s))
    P.sync()
    for x, (wa, wb), (acc, _) in zip(xs, ws, outs):
        ra, rb = oracle.poly_sums(A, x, *coefs, wa, wb)
        got = host(acc)
        assert np.array_equal(got[0], ra) and np.array_equal(got[1], rb)
    P.close()


@pytest.mark.parametrize("sched,baseline", [("steps", False), ("wave", False), ("xcd", False),
                                            ("wave", True)])
def test_time_step_graph_replays_match_eager(sched, baseline):
    A = w.anderson_3d(14)
    P = mpk.Plan(A)
    P.tune(schedule=sched, chunk_nnz=1500)
    g = np.random.default_rng(150)
    psi = dev(g.standard_normal((A.n, 4)))
    dt, M = 0.7, 12
    eager = host(P.cheb_time_step(psi, dt, M, baseline=baseline))
    out = torch.empty_like(psi)
    G = P.capture_time_step(psi, dt, M, out, baseline=baseline)
    for i in range(3):
        out.fill_(np.nan)
        torch.cuda.synchronize()
        G.launch()
        assert np.array_equal(host(out), eager), f"replay {i}"
        # unrelated eager work on the same plan between replays
        other = P.run(dev(w.uniform_vectors(A.n, 1, 160 + i)), 3)
        P.sync()
        del other
    # two steps by alternating two graphs equal two eager steps
    back = torch.empty_like(psi)
    G2 = P.capture_time_step(out, dt, M, back, baseline=baseline)
    G.launch()
    G2.launch()
    two = host(P.cheb_time_step(P.cheb_time_step(psi, dt, M, baseline=baseline), dt, M,
                                baseline=baseline))
    assert np.array_equal(host(back), two)
    G.close()
    G2.close()
    P.sync()
    P.close()


@pytest.mark.slow
def test_full_size_time_step_anderson160():
    # the benchmark's time step: 160^3 lattice, FP32 values, 4 complex states,
    # M = 16, dt = 1, original order, autotuned level-blocked and p x SpMV forms
    A, x, _, _ = w.config("anderson160_cheb16_r8")
    M, dt = 16, 1.0
    P = mpk.Plan(A, value_bits=32, reorder="none")
    xd = dev(x)
    P.autotune(xd, M, reps=1, recur=True, force=True)
    al, be, ga, wa, wb = mpk.cheb_time_coefficients(M, dt)
    ref = oracle.combine_complex(*oracle.poly_sums(A, x, al, be, ga, wa, wb, value_bits=32))
    for base in (False, True):
        out = host(P.cheb_time_step(xd, dt, M, baseline=base))
        assert np.array_equal(out, ref), base
    P.close()
