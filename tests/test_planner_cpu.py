"""Host-side tests of the C ABI: symbol exports, the planner's levels and
permutation, schedule validity and the error paths (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads as w
from tests._util import read_golden

mpk = pytest.importorskip("paper_2405_12525_amd")
from paper_2405_12525_amd import _capi  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def host_plan(A, **kw):
    kw.setdefault("device", mpk.MPK_DEVICE_NONE)
    return mpk.Plan(A, **kw)


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mpk.h")).read()
    declared = set(re.findall(r"\b(mpk_[a-z_]+)\s*\(", hdr))
    assert declared == set(_capi.EXPORTS)
    lib = _capi.load()
    for name in declared:
        assert hasattr(lib, name), name
    assert mpk.version().startswith("mpk-mi355x")


def _golden_graph():
    rows = read_golden("stencil20_graph.txt")
    n = int(rows[0][1])
    D = np.eye(n)
    for u, v in rows[1:]:
        D[int(u), int(v)] = D[int(v), int(u)] = -1.0
    return w.from_dense(D, "stencil20")


def test_planner_reproduces_paper_bfs_example():
    A = _golden_graph()
    g = read_golden("stencil20_bfs.txt")
    new_label = [int(v) for v in g[0][1:]]
    levels = [[int(v) for v in r[1:]] for r in g if r[0] == "level"]
    P = host_plan(A)
    lp, perm = P.levels()
    assert [sorted(perm[lp[i]:lp[i + 1]].tolist()) for i in range(len(lp) - 1)] == levels
    assert [perm[lp[i]:lp[i + 1]].tolist() for i in range(len(lp) - 1)] == levels  # ascending
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(A.n)
    assert iperm.tolist() == new_label


@pytest.mark.parametrize("seed,sym", [(0, True), (1, False), (2, False), (3, True)])
def test_planner_levels_match_oracle(seed, sym):
    A = w.random_sparse(400, 0.004, seed, symmetric_pattern=sym)  # often disconnected
    lv, perm_o, _ = oracle.bfs_levels(A.n, A.rowptr, A.col, root=0)
    lp, perm = host_plan(A).levels()
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(np.diff(lp), [len(L) for L in lv])


def test_planner_root_option():
    A = w.stencil_2d5(9)
    lv, perm_o, _ = oracle.bfs_levels(A.n, A.rowptr, A.col, root=40)
    lp, perm = host_plan(A, root=40).levels()
    assert np.array_equal(perm, perm_o)


@pytest.mark.parametrize("seed,sym", [(4, True), (5, False), (6, True)])
def test_planner_peripheral_root_matches_oracle(seed, sym):
    # the same George-Liu choice (an integer: exact), then the same levels
    A = w.random_sparse(300, 0.008, seed, symmetric_pattern=sym)
    r = oracle.pseudo_peripheral_root(A.n, A.rowptr, A.col)
    lv, perm_o, _ = oracle.bfs_levels(A.n, A.rowptr, A.col, root=r)
    lp, perm = host_plan(A, root="peripheral").levels()
    assert perm[0] == r
    assert np.array_equal(perm, perm_o)
    assert np.array_equal(np.diff(lp), [len(L) for L in lv])


def test_planner_peripheral_root_on_lattices():
    # a corner of the 3D 27-point stencil, and an end of a banded matrix
    A = w.stencil_3d27(7)
    lp, perm = host_plan(A, root="peripheral").levels()
    corners = {x + 7 * (y + 7 * z) for x in (0, 6) for y in (0, 6) for z in (0, 6)}
    assert perm[0] in corners and len(lp) - 1 == 7
    B = w.tridiag_1d(50)
    _, permb = host_plan(B, root="peripheral").levels()
    assert permb[0] in (0, 49)


def _level_of(lp, n):
    lev = np.empty(n, dtype=np.int64)
    for i in range(len(lp) - 1):
        lev[lp[i]:lp[i + 1]] = i
    return lev


@pytest.mark.parametrize("reorder", ["bfs", "none"])
def test_level_neighbour_property(reorder):
    # a row's neighbours lie in its own or an adjacent level (plan numbering)
    for A in (w.stencil_2d5(15), w.stencil_3d27(6), w.anderson_3d(6),
              w.random_sparse(200, 0.02, 7)):
        lp, perm = host_plan(A, reorder=reorder).levels()
        iperm = np.empty_like(perm)
        iperm[perm] = np.arange(A.n)
        lev = _level_of(lp, A.n)
        rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
        d = np.abs(lev[iperm[rows]] - lev[iperm[A.col]])
        assert d.max() <= 1
        assert sorted(perm.tolist()) == list(range(A.n))
        if reorder == "none":
            assert np.array_equal(perm, np.arange(A.n))


def _check_schedule(A, s, p):
    """Every (chunk, power) once; dependencies strictly earlier (in issue order,
    or in an earlier launch for the one-launch-per-diagonal schedule)."""
    cp, lo, hi, tasks = s["chunk_ptr"], s["dep_lo"], s["dep_hi"], s["tasks"]
    nc = len(cp) - 1
    assert cp[0] == 0 and cp[-1] == A.n and np.all(np.diff(cp) > 0)
    assert tasks.shape == (nc * p, 2)
    sp = s["step_ptr"]
    assert sp[0] == 0 and sp[-1] == len(tasks) and np.all(np.diff(sp) >= 0)
    launch = np.repeat(np.arange(len(sp) - 1), np.diff(sp))
    when = -np.ones((p + 1, nc), dtype=np.int64)
    for t, (c, k) in enumerate(tasks):
        assert when[k, c] < 0
        when[k, c] = launch[t] if len(sp) > 2 else t
    assert (when[1:] >= 0).all()
    for c in range(nc):
        assert lo[c] <= c <= hi[c]
        for k in range(2, p + 1):
            assert when[k - 1, lo[c]:hi[c] + 1].max() < when[k, c]


def _deps_cover_reads(A, P, s):
    """Every column a chunk's rows read lies in its dependency range."""
    lp, perm = P.levels()
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(A.n)
    cp = s["chunk_ptr"]
    chunk_of = np.repeat(np.arange(len(cp) - 1), np.diff(cp))
    for new in range(A.n):
        old = perm[new]
        cols = iperm[A.col[A.rowptr[old]:A.rowptr[old + 1]]]
        c = chunk_of[new]
        if cols.size:
            assert chunk_of[cols].min() >= s["dep_lo"][c]
            assert chunk_of[cols].max() <= s["dep_hi"][c]


@pytest.mark.parametrize("sched", ["steps", "wave", "diag", "powers"])
@pytest.mark.parametrize("reorder", ["bfs", "none"])
def test_schedules_are_topological(sched, reorder):
    for A in (w.stencil_2d5(30), w.random_sparse(300, 0.01, 3), w.anderson_3d(7)):
        P = host_plan(A, reorder=reorder)
        P.tune(schedule=sched, chunk_nnz=64, cache_bytes=20000, cache_safety=1.0, lag=0)
        for p in (1, 2, 5):
            s = P.schedule(p)
            _check_schedule(A, s, p)
            _deps_cover_reads(A, P, s)


def _check_xcd_schedule(A, P, s, p):
    """XCD schedule: every chunk boundary on a multiple of 16 rows (line
    closed) and each chunk inside the aligned span of one level (from its
    first row rounded up to a multiple of 16 to the next level's), exact
    dependency lists, every (chunk, power) once in its owner's queue,
    write-back flags exactly where a consumer lives in another queue, and the
    queues drain with one worker each (no cross-queue deadlock)."""
    cp, tasks, qp = s["chunk_ptr"], s["tasks"], s["qptr"]
    dp, di, cx, ro = s["dep_ptr"], s["dep_idx"], s["chunk_xcd"], s["remote_out"]
    nc, nq = len(cp) - 1, s["n_queues"]
    lp, perm = P.levels()
    assert cp[0] == 0 and cp[-1] == A.n and np.all(np.diff(cp) > 0)
    assert np.all(cp[1:-1] % 16 == 0)
    span = np.minimum(A.n, (lp + 15) // 16 * 16)
    span[-1] = A.n
    level = np.searchsorted(span, cp[:-1], side="right") - 1
    assert np.array_equal(level, s["chunk_group"])
    assert np.all(cp[1:] <= span[level + 1])
    # exact lists: the chunks the rows read, plus the chunk itself
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(A.n)
    chunk_of = np.repeat(np.arange(nc), np.diff(cp))
    for c in range(nc):
        want = {c}
        for new in range(cp[c], cp[c + 1]):
            old = perm[new]
            want |= set(chunk_of[iperm[A.col[A.rowptr[old]:A.rowptr[old + 1]]]].tolist())
        assert di[dp[c]:dp[c + 1]].tolist() == sorted(want)
    # write-back flags
    want_ro = np.zeros(nc, np.int32)
    for c in range(nc):
        for d in di[dp[c]:dp[c + 1]]:
            if cx[d] != cx[c]:
                want_ro[d] = 1
    if nq == 1:
        assert ro.all()  # one queue: no binding to an XCD, every result is written back
    else:
        assert np.array_equal(ro, want_ro)
    # queues
    assert qp[0] == 0 and qp[-1] == nc * p and len(qp) == nq + 1
    seen = set()
    for q in range(nq):
        last = {}
        for c, k in tasks[qp[q]:qp[q + 1]]:
            assert cx[c] == q and (c, k) not in seen and last.get(c, 0) == k - 1
            seen.add((c, k))
            last[c] = k
    assert len(seen) == nc * p
    # one worker per queue, each blocked until its head task's inputs are done
    done = np.zeros(nc, np.int64)
    head = qp[:-1].copy()
    left = nc * p
    while left:
        moved = False
        for q in range(nq):
            if head[q] < qp[q + 1]:
                c, k = tasks[head[q]]
                if all(done[d] >= k - 1 for d in di[dp[c]:dp[c + 1]]):
                    done[c] = k
                    head[q] += 1
                    left -= 1
                    moved = True
        assert moved, "queues deadlock"


@pytest.mark.parametrize("reorder", ["bfs", "none"])
def test_xcd_schedule_lists_queues_and_progress(reorder):
    for A in (w.stencil_2d5(30), w.random_sparse(300, 0.01, 3), w.anderson_3d(7),
              w.stencil_3d27(12)):
        P = host_plan(A, reorder=reorder)
        for chunk in (64, 4096):
            P.tune(schedule="xcd", chunk_nnz=chunk, cache_bytes=20000, lag=0)
            for p in (1, 2, 5):
                s = P.schedule(p)
                assert s["n_queues"] == 8
                _check_xcd_schedule(A, P, s, p)


def test_xcd_chunks_start_on_16_row_boundaries():
    A = w.stencil_3d27(23)   # n = 12167: not a multiple of 16
    P = host_plan(A)
    P.tune(schedule="xcd", chunk_nnz=2000)
    s = P.schedule(4)
    cp = s["chunk_ptr"]
    assert cp[-1] == A.n and all(r % 16 == 0 for r in cp[:-1].tolist())


def test_xcd_schedule_with_few_workgroups_uses_one_queue():
    A = w.stencil_2d5(40)
    P = host_plan(A)
    P.tune(schedule="xcd", workgroups=4, chunk_nnz=100)
    s = P.schedule(3)
    assert s["n_queues"] == 1 and s["remote_out"].all()
    _check_xcd_schedule(A, P, s, 3)


def test_diag_schedule_is_the_papers_lp_order():
    # a path graph has one vertex per BFS level; one chunk per level and one
    # level per group turn the chunk schedule into the Lp diagram of Fig. lp_basic
    grid = [[int(v) for v in r[1:]] for r in read_golden("lp_order_10x5.txt")]
    A = w.tridiag_1d(10)
    P = host_plan(A)
    P.tune(schedule="diag", cache_bytes=1, cache_safety=1.0, chunk_nnz=1)
    s = P.schedule(5)
    assert s["n_groups"] == 10 and s["n_chunks"] == 10
    for step, (c, k) in enumerate(s["tasks"]):
        assert grid[k - 1][c] == step
    assert list(map(tuple, s["tasks"])) == [(i, p) for i, p in oracle.lp_diagonal_order(10, 5)]


def test_steps_schedule_diagonals():
    # one vertex per level and per group: launch d holds (g, k) with g + 2(k-1) = d
    A = w.tridiag_1d(12)
    P = host_plan(A)
    P.tune(schedule="steps", cache_bytes=1, cache_safety=1.0, chunk_nnz=1)
    s = P.schedule(4)
    assert s["n_groups"] == 12 and s["n_steps"] == 12 + 2 * 3
    sp = s["step_ptr"]
    for d in range(s["n_steps"]):
        got = sorted(map(tuple, s["tasks"][sp[d]:sp[d + 1]]))
        want = sorted((d - 2 * (k - 1), k) for k in range(1, 5) if 0 <= d - 2 * (k - 1) < 12)
        assert got == want
    _check_schedule(A, s, 4)


def test_wave_lag_changes_order_not_validity():
    A = w.stencil_2d5(40)
    P = host_plan(A, reorder="none")
    orders = []
    for lag in (1, 3, 50):
        P.tune(schedule="wave", chunk_nnz=40, lag=lag)
        s = P.schedule(4)
        _check_schedule(A, s, 4)
        assert s["lag"] == lag
        orders.append(s["tasks"].tolist())
    assert orders[0] != orders[2]


def test_plan_info_fields():
    A = w.stencil_3d27(5)
    P = host_plan(A, value_bits=32)
    i = P.info()
    assert i["n"] == A.n and i["nnz"] == A.nnz and i["value_bits"] == 32
    assert i["matrix_bytes"] == 4 * (A.n + 1) + 8 * A.nnz
    assert i["n_levels"] == 5  # cube shells max(x,y,z) = const from the corner


# ------------------------------------------------------------------ error paths

def _raw_plan(n, rowptr, col, val, device=mpk.MPK_DEVICE_NONE):
    L = _capi.load()
    rowptr = np.asarray(rowptr, np.int32)
    col = np.asarray(col, np.int32)
    val = np.asarray(val, np.float64)
    csr = _capi.CSRStruct(n, int(rowptr[-1]) if rowptr.size else 0, rowptr.ctypes.data,
                          col.ctypes.data, val.ctypes.data)
    opts = _capi.PlanOpts()
    L.mpk_plan_opts_default(ctypes.byref(opts))
    opts.device = device
    h = ctypes.c_void_p()
    st = L.mpk_plan(ctypes.byref(csr), ctypes.byref(opts), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("rowptr,col,status", [
    ([0, 2, 1, 3], [0, 1, 2], _capi.MPK_EBADCSR),      # decreasing rowptr
    ([1, 2, 3, 3], [0, 1, 2], _capi.MPK_EBADCSR),      # rowptr[0] != 0
    ([0, 1, 2, 3], [0, 3, 2], _capi.MPK_EBADCSR),      # column out of range
    ([0, 1, 2, 3], [0, -1, 2], _capi.MPK_EBADCSR),     # negative column
])
def test_bad_csr_rejected(rowptr, col, status):
    st, h = _raw_plan(3, rowptr, col, np.ones(3))
    assert st == status
    assert not h.value
    assert _capi.load().mpk_last_error()


def test_run_argument_errors_without_device():
    A = w.stencil_2d5(4)
    P = host_plan(A)
    L = _capi.load()
    assert L.mpk_run(P._h, None, 0, 1, None, None) == _capi.MPK_EINVAL
    assert L.mpk_run(P._h, None, 3, 17, None, None) == _capi.MPK_EUNSUPPORTED
    assert L.mpk_run(P._h, None, 3, 1, None, None) == _capi.MPK_ENODEVICE
    assert L.mpk_run_baseline(P._h, None, -1, 1, None, None) == _capi.MPK_EINVAL
    assert L.mpk_run(None, None, 3, 1, None, None) == _capi.MPK_EINVAL
    assert L.mpk_plan_sync(P._h) == _capi.MPK_ENODEVICE
    assert L.mpk_plan_prepare(P._h, 0, 1) == _capi.MPK_EINVAL
    assert L.mpk_plan_prepare(P._h, 3, 17) == _capi.MPK_EUNSUPPORTED
    assert L.mpk_plan_prepare(P._h, 3, 1) == _capi.MPK_ENODEVICE
    assert L.mpk_plan_prepare(None, 3, 1) == _capi.MPK_EINVAL


def test_tune_validation():
    P = host_plan(w.stencil_2d5(4))
    with pytest.raises(mpk.MPKError):
        P.tune(cache_safety=0.0)
    with pytest.raises(mpk.MPKError):
        P.tune(schedule=7)
    with pytest.raises(mpk.MPKError):
        P.tune(chunk_nnz=0)
    with pytest.raises(mpk.MPKError):
        P.tune(seg_powers=65)
    with pytest.raises(mpk.MPKError):
        P.tune(skip_ahead=9)
    with pytest.raises(mpk.MPKError):
        P.tune(seg_powers=-1)
    with pytest.raises(mpk.MPKError):
        mpk.Plan(w.stencil_2d5(4), device=mpk.MPK_DEVICE_NONE, value_bits=16)
    with pytest.raises(mpk.MPKError):
        mpk.Plan(w.stencil_2d5(4), device=mpk.MPK_DEVICE_NONE, root=16)


def test_empty_and_tiny_plans():
    A = w.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    P = host_plan(A)
    assert P.info()["n"] == 0
    s = P.schedule(3)
    assert s["n_chunks"] == 0 and s["n_tasks"] == 0
    B = w.identity(1)
    s = host_plan(B).schedule(4)
    assert s["n_chunks"] == 1 and s["tasks"].tolist() == [[0, 1], [0, 2], [0, 3], [0, 4]]


# ------------------------------------------------------------------ sub-levels and budgets

@pytest.mark.parametrize("which", ["paper20", "grid2d", "cube", "rand", "rand_nonsym"])
def test_sublevel_order_matches_oracle(which):
    A = {"paper20": _golden_graph, "grid2d": lambda: w.stencil_2d5(17),
         "cube": lambda: w.stencil_3d27(9), "rand": lambda: w.random_sparse(300, 0.01, 4),
         "rand_nonsym": lambda: w.random_sparse(300, 0.01, 5, symmetric_pattern=False)}[which]()
    P = host_plan(A, reorder="sublevels")
    lp, perm = P.levels()
    d1, d2, operm, _ = oracle.sublevels(A.n, A.rowptr, A.col, 0)
    assert np.array_equal(perm, operm)
    assert [int(v) for v in lp] == [0] + np.cumsum(np.bincount(d1)).tolist()
    info = P.info()
    assert info["sublevel_root"] == oracle.sublevel_root(A.n, A.rowptr, A.col, 0)
    assert info["max_sublevels"] == max(len(set(d2[d1 == i].tolist())) for i in range(d1.max() + 1))
    # the same levels as the plain BFS order, only reordered inside each level
    lpb, permb = host_plan(A).levels()
    assert np.array_equal(lp, lpb)
    for i in range(len(lp) - 1):
        assert sorted(perm[lp[i]:lp[i + 1]].tolist()) == permb[lp[i]:lp[i + 1]].tolist()


def test_sublevel_order_with_given_second_root():
    A = w.stencil_2d5(12)
    P = host_plan(A, reorder="sublevels", sublevel_root=5)
    _, perm = P.levels()
    assert np.array_equal(perm, oracle.sublevels(A.n, A.rowptr, A.col, 0, root2=5)[2])
    assert P.info()["sublevel_root"] == 5
    with pytest.raises(mpk.MPKError):
        host_plan(A, reorder="sublevels", sublevel_root=A.n)


@pytest.mark.parametrize("sched", ["steps", "wave", "diag", "powers"])
def test_schedules_on_sublevel_order_are_topological(sched):
    for A in (w.stencil_3d27(10), w.random_sparse(300, 0.01, 3)):
        P = host_plan(A, reorder="sublevels")
        P.tune(schedule=sched, chunk_nnz=200, cache_bytes=40000, lag=0)
        for p in (1, 4):
            s = P.schedule(p)
            _check_schedule(A, s, p)
            _deps_cover_reads(A, P, s)


def test_xcd_schedule_on_sublevel_order():
    for A in (w.stencil_3d27(12), w.anderson_3d(8)):
        P = host_plan(A, reorder="sublevels")
        P.tune(schedule="xcd", chunk_nnz=300, lag=0)
        for p in (2, 5):
            s = P.schedule(p)
            _check_xcd_schedule(A, P, s, p)


def test_planner_budget_options():
    A = w.stencil_3d27(14)
    d = host_plan(A).info()
    assert d["l2_bytes"] == 4 << 20 and d["mall_bytes"] == 64 << 20 and d["min_group_rows"] == 0
    P = host_plan(A, l2_bytes=1 << 20, mall_bytes=8 << 20, min_group_rows=600)
    i = P.info()
    assert (i["l2_bytes"], i["mall_bytes"], i["min_group_rows"]) == (1 << 20, 8 << 20, 600)
    assert P.tuning["cache_bytes"] == 8 << 20          # the plan's budget C
    # every level group but the last holds at least min_group_rows rows
    P.tune(schedule="steps", cache_bytes=20000, chunk_nnz=1 << 20)
    lp, _ = P.levels()
    s = P.schedule(3)
    cp = np.asarray(s["chunk_ptr"])
    grp = np.asarray(s["chunk_group"])
    rows = np.bincount(grp, weights=np.diff(cp))
    assert rows[:-1].min() >= 600
    Q = host_plan(A)
    Q.tune(schedule="steps", cache_bytes=20000, chunk_nnz=1 << 20)
    assert Q.schedule(3)["n_groups"] > s["n_groups"]
    # the L2 budget bounds the XCD schedule's chunks: p + 1 of them fit it
    for l2 in (1 << 20, 64 << 10):
        R = host_plan(A, l2_bytes=l2)
        R.tune(schedule="xcd", chunk_nnz=1 << 20)
        sx = R.schedule(4)
        cp = np.asarray(sx["chunk_ptr"])
        _, perm = R.levels()
        prp = np.concatenate([[0], np.cumsum(np.diff(A.rowptr)[perm])])  # plan-order rowptr
        nz = prp[cp[1:]] - prp[cp[:-1]]
        # a chunk ends on the row that reaches the cap, rounded to 16 rows
        assert nz.max() <= max(1024, l2 // (5 * 12)) + 27 * 16
    for bad in (dict(l2_bytes=-1), dict(mall_bytes=1000), dict(min_group_rows=-3)):
        with pytest.raises(mpk.MPKError):
            host_plan(A, **bad)


def test_fingerprint_keys_pattern_and_options():
    """The matrix part of the autotuner's cache key: equal for the same
    pattern and ordering options (values do not change the tuning; the value
    precision is a key field of its own), different for another pattern, row
    order or root."""
    A = w.stencil_3d27(8)
    B = w.CSR(A.n, A.rowptr, A.col, A.val * 2.0 + 1.0, "scaled")
    C = w.anderson_3d(8)
    fp = lambda M, **kw: mpk.Plan(M, device=mpk.MPK_DEVICE_NONE, **kw).info()["fingerprint"]
    assert fp(A) == fp(A) == fp(B) == fp(A, value_bits=32)
    assert fp(A) != fp(C)
    assert fp(A) != fp(A, reorder="none")
    assert fp(A) != fp(A, root=5)
