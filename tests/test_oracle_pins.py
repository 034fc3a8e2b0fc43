"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formula: every expected value comes from a
closed form, an exact-integer or exact-rational brute force, a library routine
of a different kind (dense matrix power, graph distances), or a worked example
printed in the paper (tests/golden/).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
import workloads as w
from tests._util import read_golden, rel_err_per_power


# ------------------------------------------------------------------ exact results

def test_identity_powers_are_exact():
    A = w.identity(37)
    x = w.uniform_vectors(37, 3, 7)
    Y = oracle.powers(A, x, 5)
    for k in range(5):
        assert np.array_equal(Y[k], x)


def test_permutation_powers_are_exact_and_not_transposed():
    # (P x)[i] = x[sigma[i]]; P^k composes the index map k times.
    P, sigma = w.permutation_matrix(50, 11)
    x = w.uniform_vectors(50, 2, 3)
    Y = oracle.powers(P, x, 6)
    idx = np.arange(50)
    for k in range(6):
        idx = sigma[idx]
        assert np.array_equal(Y[k], x[idx])
    # the transpose would apply sigma^{-1}: make sure that differs here
    inv = np.argsort(sigma)
    assert not np.array_equal(Y[0], x[inv])


def test_laplacian_1d_delta_binomials():
    # tridiag(-1, 2, -1) applied k times to a delta gives (-1)^j C(2k, k+j)
    n, c = 121, 60
    A = w.tridiag_1d(n)
    x = np.zeros((n, 1))
    x[c, 0] = 1.0
    p = 24
    Y = oracle.powers(A, x, p)
    for k in range(1, p + 1):
        expect = np.zeros(n)
        for j in range(-k, k + 1):
            expect[c + j] = (-1) ** j * math.comb(2 * k, k + j)
        assert np.array_equal(Y[k - 1, :, 0], expect), k


def _exact_int_powers(A, xi, p):
    """A^k x in exact integer arithmetic through a dense int64 matrix."""
    D = A.to_dense()
    Di = D.astype(np.int64)
    assert np.array_equal(Di.astype(np.float64), D)
    out, y = [], xi.astype(np.int64)
    for _ in range(p):
        y = Di @ y
        out.append(y.copy())
    return np.stack(out)


@pytest.mark.parametrize("A,p", [(w.stencil_2d5(12), 7), (w.stencil_3d27(6), 6),
                                 (w.random_sparse(40, 0.1, 5, values="int"), 6)])
def test_integer_inputs_exact(A, p):
    x = w.integer_vectors(A.n, 2, 99)
    Y = oracle.powers(A, x, p)
    E = _exact_int_powers(A, x, p)
    assert np.abs(E).max() < 2 ** 53
    assert np.array_equal(Y, E.astype(np.float64))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dense_brute_force_nonsymmetric(seed):
    A = w.random_sparse(48, 0.12, seed)
    x = w.uniform_vectors(48, 3, seed + 100)
    p = 6
    D = A.to_dense()
    ref = np.stack([np.linalg.matrix_power(D, k) @ x for k in range(1, p + 1)])
    assert rel_err_per_power(oracle.powers(A, x, p), ref).max() < 1e-12
    # a transposed operand would be caught here
    refT = np.stack([np.linalg.matrix_power(D.T, k) @ x for k in range(1, p + 1)])
    assert rel_err_per_power(refT, ref).max() > 1e-3


def test_fp32_values_round_then_promote():
    A = w.random_sparse(60, 0.1, 4)
    x = w.uniform_vectors(60, 2, 5)
    Y32 = oracle.powers(A, x, 5, value_bits=32)
    A2 = w.CSR(A.n, A.rowptr, A.col, A.val.astype(np.float32).astype(np.float64))
    assert np.array_equal(Y32, oracle.powers(A2, x, 5))
    assert rel_err_per_power(Y32, oracle.powers(A, x, 5)).max() < 1e-5


# ------------------------------------------------------------------ recurrence

def test_chebyshev_on_diagonal_is_cos_k_theta():
    th = np.linspace(0.05, 3.1, 30)
    n = th.size
    A = w.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.cos(th))
    x = w.uniform_vectors(n, 1, 8)
    p = 16
    Y = oracle.recur(A, x, *oracle.chebyshev_coefficients(p))
    for k in range(1, p + 1):
        np.testing.assert_allclose(Y[k - 1, :, 0], np.cos(k * th) * x[:, 0], rtol=0, atol=1e-13)


def test_chebyshev_fourier_mode_periodic_hopping():
    # H = (S + S^-1)/2 on a ring: v_j = cos(theta_m j) has eigenvalue cos(theta_m)
    n, m = 64, 5
    A = w.tridiag_1d(n, diag=0.0, off=0.5, periodic=True)
    th = 2 * math.pi * m / n
    v = np.cos(th * np.arange(n)).reshape(n, 1)
    p = 12
    Yc = oracle.recur(A, v, *oracle.chebyshev_coefficients(p))
    Yp = oracle.powers(A, v, p)
    for k in range(1, p + 1):
        np.testing.assert_allclose(Yc[k - 1], math.cos(k * th) * v, atol=1e-13)
        np.testing.assert_allclose(Yp[k - 1], math.cos(th) ** k * v, atol=1e-13)


def test_general_recurrence_exact_rationals():
    # dyadic data keeps every intermediate exactly representable; the
    # expected values come from a Fraction brute force over a dense matrix.
    D = np.array([[0.5, -1.0, 0.0, 0.25],
                  [0.0, 1.0, 0.5, 0.0],
                  [-0.25, 0.0, -0.5, 1.0],
                  [1.0, 0.0, 0.0, 0.5]])
    A = w.from_dense(D)
    x = np.array([[1.0, -2.0], [0.5, 1.0], [-1.0, 0.0], [2.0, 0.25]])
    alpha = np.array([1.0, 2.0, -0.5, 1.0, 2.0, 0.5])
    beta = np.array([0.5, 0.0, 1.0, -1.0, 0.25, 0.0])
    gamma = np.array([0.0, -1.0, 0.5, 0.25, -1.0, 2.0])
    Y = oracle.recur(A, x, alpha, beta, gamma)
    F = [[Fraction(v) for v in row] for row in D]
    X = [[Fraction(v) for v in row] for row in x]
    prev, cur, out = None, X, []
    for j in range(alpha.size):
        t = [[sum(F[i][c] * cur[c][r] for c in range(4)) for r in range(2)] for i in range(4)]
        nxt = [[Fraction(alpha[j]) * t[i][r] + Fraction(beta[j]) * cur[i][r]
                + (Fraction(gamma[j]) * prev[i][r] if prev is not None else 0)
                for r in range(2)] for i in range(4)]
        out.append(nxt)
        prev, cur = cur, nxt
    assert np.array_equal(Y, np.array(out, dtype=np.float64))


# ------------------------------------------------------------------ invariants

def test_split_and_block_invariants():
    A = w.stencil_2d5(20)
    x = w.uniform_vectors(A.n, 4, 21)
    Y = oracle.powers(A, x, 7)
    Ya = oracle.powers(A, x, 3)
    Yb = oracle.powers(A, Ya[-1], 4)
    assert np.array_equal(Y[:3], Ya) and np.array_equal(Y[3:], Yb)
    for r in range(4):
        assert np.array_equal(Y[:, :, r:r + 1], oracle.powers(A, x[:, r:r + 1], 7))
    # linearity
    Z = oracle.powers(A, 2.0 * x[:, :1] - 3.0 * x[:, 1:2], 7)
    assert rel_err_per_power(Z, 2.0 * Y[:, :, :1] - 3.0 * Y[:, :, 1:2]).max() < 1e-13


def test_empty_matrix():
    A = w.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert oracle.powers(A, np.zeros((0, 1)), 3).shape == (3, 0, 1)


# ------------------------------------------------------------------ levels and order

def _golden_graph():
    rows = read_golden("stencil20_graph.txt")
    n = int(rows[0][1])
    D = np.eye(n)
    for u, v in rows[1:]:
        D[int(u), int(v)] = D[int(v), int(u)] = -1.0
    return w.from_dense(D, "stencil20")


def test_paper_stencil_levels_and_permutation():
    A = _golden_graph()
    g = read_golden("stencil20_bfs.txt")
    new_label = [int(v) for v in g[0][1:]]
    levels = [[int(v) for v in r[1:]] for r in g if r[0] == "level"]
    row8 = [int(v) for v in g[-1][1:]]
    assert list(A.col[A.rowptr[8]:A.rowptr[9]]) == row8
    lv, perm, iperm = oracle.bfs_levels(A.n, A.rowptr, A.col, root=0)
    assert lv == levels
    assert list(iperm) == new_label


def test_lp_diagram_order_matches_figure():
    grid = [[int(v) for v in r[1:]] for r in read_golden("lp_order_10x5.txt")]
    order = oracle.lp_diagonal_order(10, 5)
    assert len(order) == 50
    for step, (i, p) in enumerate(order):
        assert grid[p - 1][i] == step
    assert grid[0][5] == 15 and grid[1][5] == 21  # stated next to the figure


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_levels_are_graph_distances(seed):
    A = w.random_sparse(300, 0.008, seed, symmetric_pattern=False)
    lv, perm, iperm = oracle.bfs_levels(A.n, A.rowptr, A.col, root=0)
    M = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(A.n, A.n))
    dist = csg.shortest_path(M, unweighted=True, directed=False, indices=0)
    comp0 = [v for v in range(A.n) if np.isfinite(dist[v])]
    lev_of = {v: i for i, L in enumerate(lv) for v in L}
    for v in comp0:
        assert lev_of[v] == dist[v]
    # every vertex appears exactly once; neighbours are at most one level apart
    assert sorted(perm.tolist()) == list(range(A.n))
    for v in range(A.n):
        for e in range(A.rowptr[v], A.rowptr[v + 1]):
            assert abs(lev_of[v] - lev_of[int(A.col[e])]) <= 1


def test_permute_csr_symmetric():
    A = w.random_sparse(30, 0.2, 9)
    perm = w.rng(1).permutation(30)
    B = oracle.permute_csr(A, perm)
    D, E = A.to_dense(), B.to_dense()
    assert np.array_equal(E, D[np.ix_(perm, perm)])


def test_zero_coefficient_omits_its_term():
    # row 0 is empty, so (A x)[0] = 0 exactly; x[0] = inf.  With beta = 0 the
    # beta term is absent (finite result); with beta != 0 it is inf.
    A = w.CSR(2, np.array([0, 0, 1], np.int32), np.array([1], np.int32), np.array([2.0]), "t")
    x = np.array([[np.inf], [1.0]])
    Y = oracle.recur(A, x, [3.0], [0.0], [0.0])
    assert Y[0, 0, 0] == 0.0 and Y[0, 1, 0] == 6.0
    Y = oracle.recur(A, x, [3.0], [1.0], [0.0])
    assert np.isinf(Y[0, 0, 0]) and Y[0, 1, 0] == 7.0


# ------------------------------------------------- polynomial sums (time step)

def test_poly_single_weight_selects_one_vector():
    A = w.stencil_2d5(9)
    x = w.uniform_vectors(A.n, 2, 31)
    al, be, ga = oracle.chebyshev_coefficients(6)
    Y = oracle.recur(A, x, al, be, ga)
    for k in range(7):
        wa = np.zeros(7)
        wa[k] = 1.0
        acc, none = oracle.poly_sums(A, x, al, be, ga, wa)
        assert none is None
        assert np.array_equal(acc, x if k == 0 else Y[k - 1]), k
    zero, _ = oracle.poly_sums(A, x, al, be, ga, np.zeros(7))
    assert np.array_equal(zero, np.zeros_like(x))


def test_poly_integer_weights_on_laplacian_binomials():
    # plain powers of tridiag(-1, 2, -1) on a delta are (-1)^j C(2k, k+j);
    # integer weights keep every partial sum an exact integer
    n, c, p = 81, 40, 18
    A = w.tridiag_1d(n)
    x = np.zeros((n, 1))
    x[c, 0] = 1.0
    wts = np.array([(k % 5) - 2 for k in range(p + 1)], dtype=np.float64)
    acc, _ = oracle.poly_sums(A, x, np.ones(p), np.zeros(p), np.zeros(p), wts)
    expect = np.zeros(n)
    expect[c] = wts[0]
    for k in range(1, p + 1):
        for j in range(-k, k + 1):
            expect[c + j] += wts[k] * (-1) ** j * math.comb(2 * k, k + j)
    assert np.array_equal(acc[:, 0], expect)


def test_bessel_weights_textbook_values():
    # J_0(1) and J_1(1) from Abramowitz & Stegun, Table 9.1
    al, be, ga, wa, wb = oracle.cheb_time_coefficients(4, 1.0)
    assert abs(wa[0] - 0.7651976865579666) < 1e-15
    assert abs(wb[1] + 2 * 0.4400505857449335) < 1e-15
    # (-i)^k: real at even k (sign +, -, ...), imaginary at odd k (-, +, ...)
    assert wb[0] == 0 and wa[1] == 0 and wb[2] == 0 and wa[3] == 0 and wb[4] == 0
    assert wa[2] < 0 and wb[3] > 0 and wa[4] > 0
    assert np.array_equal(al, [1, 2, 2, 2]) and not be.any() and np.array_equal(ga, [0, -1, -1, -1])


def _complex_pairs(z):
    out = np.empty((z.shape[0], 2 * z.shape[1]))
    out[:, 0::2] = z.real
    out[:, 1::2] = z.imag
    return out


def test_time_step_on_diagonal_is_jacobi_anger():
    # for H = diag(cos th) the step is exp(-i dt cos th) psi (Jacobi-Anger);
    # truncation after M = 30 at dt = 2.5 leaves < 1e-20
    th = np.linspace(0.0, math.pi, 41)
    n = th.size
    A = w.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.cos(th))
    g = np.random.default_rng(77)
    psi = g.standard_normal((n, 2)) + 1j * g.standard_normal((n, 2))
    out = oracle.cheb_time_step(A, _complex_pairs(psi), 2.5, 30)
    expect = np.exp(-1j * 2.5 * np.cos(th))[:, None] * psi
    np.testing.assert_allclose(out, _complex_pairs(expect), rtol=0, atol=1e-13)


def test_time_step_dense_matches_matrix_exponential():
    from scipy.linalg import expm
    g = np.random.default_rng(78)
    n = 40
    B = g.standard_normal((n, n)) * (g.random((n, n)) < 0.2)
    H = (B + B.T) / 2
    H /= np.abs(H).sum(axis=1).max()          # Gershgorin: spectrum in [-1, 1]
    A = w.from_dense(H)
    psi = g.standard_normal((n, 1)) + 1j * g.standard_normal((n, 1))
    out = oracle.cheb_time_step(A, _complex_pairs(psi), 1.7, 40)
    expect = expm(-1j * 1.7 * H) @ psi
    np.testing.assert_allclose(out, _complex_pairs(expect), rtol=0, atol=1e-12)
    # a unitary step keeps the norm
    z = out[:, 0] + 1j * out[:, 1]
    assert abs(np.linalg.norm(z) - np.linalg.norm(psi)) < 1e-12


# ------------------------------------------------------------ root selection

def _ecc(N, r):
    seen, front, depth = {r}, {r}, 0
    while True:
        nxt = {v for u in front for v in N[u]} - seen
        if not nxt:
            return depth
        seen |= nxt
        front = nxt
        depth += 1


def _csr_from_edges(n, edges):
    d = np.zeros((n, n))
    for a, b in edges:
        d[a, b] = d[b, a] = 1.0
    for i in range(n):
        d[i, i] = 4.0
    return w.from_dense(d)


@pytest.mark.parametrize("seed", range(8))
def test_peripheral_root_of_a_tree_ends_a_diameter(seed):
    # on a tree, a farthest vertex from any vertex ends a longest path, so
    # the root's eccentricity is the tree's diameter (brute force over all)
    g = np.random.default_rng(300 + seed)
    n = int(g.integers(5, 60))
    edges = [(i, int(g.integers(0, i))) for i in range(1, n)]
    A = _csr_from_edges(n, edges)
    r = oracle.pseudo_peripheral_root(n, A.rowptr, A.col)
    N = oracle.neighbour_sets(n, A.rowptr, A.col)
    assert _ecc(N, r) == max(_ecc(N, v) for v in range(n))


def test_peripheral_root_of_a_scrambled_path_is_an_end():
    n = 31
    order = np.random.default_rng(9).permutation(n)      # path visits order[0], order[1], ...
    edges = [(int(order[i]), int(order[i + 1])) for i in range(n - 1)]
    A = _csr_from_edges(n, edges)
    r = oracle.pseudo_peripheral_root(n, A.rowptr, A.col)
    assert r in (int(order[0]), int(order[-1]))


def test_peripheral_root_of_a_grid_is_a_corner():
    A = w.stencil_2d5(9)      # 9 x 9 grid, row 0 is a corner
    for start in (40, 13, 0):
        r = oracle.pseudo_peripheral_root(A.n, A.rowptr, A.col, start=start)
        assert r in (0, 8, 72, 80), (start, r)


# ------------------------------------------------------------------ sub-levels
# (levels broken into sub-levels by a second breadth-first distance; the
# paper names the recursion stage s_m in Sec. "Experimental Setup" but gives
# no construction, so these pin the reading the oracle states)

def _coords(v, L):
    return v % L, (v // L) % L, v // (L * L)


@pytest.mark.parametrize("L", [5, 8])
def test_sublevels_of_a_2d_grid_are_manhattan_coordinates(L):
    # 5-point grid, root at the corner (0, 0): the levels are the
    # anti-diagonals x + y, the widest is x + y = L - 1, its smallest vertex
    # (L-1, 0) is farthest from (0, L-1); distances are Manhattan
    A = w.stencil_2d5(L)
    assert oracle.sublevel_root(A.n, A.rowptr, A.col, 0) == (L - 1) * L
    d1, d2, perm, iperm = oracle.sublevels(A.n, A.rowptr, A.col, 0)
    for v in range(A.n):
        x, y, _ = _coords(v, L)
        assert d1[v] == x + y and d2[v] == x + (L - 1 - y), v


@pytest.mark.parametrize("L", [4, 6])
def test_sublevels_of_a_27_point_cube_are_chebyshev_shells(L):
    # 27-point stencil: graph distance = Chebyshev distance; levels from the
    # corner are the shells max(x, y, z); the widest is the outer shell,
    # whose smallest vertex (L-1, 0, 0) is at distance L - 1 from
    # (0, L-1, 0), the smallest vertex of the shell at that distance
    A = w.stencil_3d27(L)
    r2 = oracle.sublevel_root(A.n, A.rowptr, A.col, 0)
    assert _coords(r2, L) == (0, L - 1, 0)
    d1, d2, _, _ = oracle.sublevels(A.n, A.rowptr, A.col, 0)
    for v in range(A.n):
        x, y, z = _coords(v, L)
        assert d1[v] == max(x, y, z) and d2[v] == max(x, L - 1 - y, z), v


def _random_connected(n, deg, seed, symmetric=True):
    g = np.random.default_rng(seed)
    D = np.eye(n)
    for v in range(1, n):              # a random spanning tree keeps it connected
        D[v, g.integers(0, v)] = -1.0
    for _ in range(n * deg):
        a, b = g.integers(0, n, 2)
        D[a, b] = -1.0
    if symmetric:
        D = np.minimum(D, D.T)
    return w.from_dense(D, f"rand{seed}")


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("symmetric", [True, False])
def test_sublevel_distances_match_graph_distances(seed, symmetric):
    A = _random_connected(60, 2, seed, symmetric)
    M = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(A.n, A.n))
    root = int(np.random.default_rng(seed).integers(0, A.n))
    r2 = oracle.sublevel_root(A.n, A.rowptr, A.col, root)
    d1, d2, _, _ = oracle.sublevels(A.n, A.rowptr, A.col, root)
    # G(A) ignores edge direction (the pattern is symmetrised for levels)
    assert np.array_equal(d1, csg.shortest_path(M, unweighted=True, directed=False, indices=root))
    assert np.array_equal(d2, csg.shortest_path(M, unweighted=True, directed=False, indices=r2))
    # the second root lies in the first widest level and is farthest there
    # from that level's smallest vertex
    widths = np.bincount(d1)
    W = np.flatnonzero(d1 == int(np.argmax(widths)))
    dw = csg.shortest_path(M, unweighted=True, directed=False, indices=int(W[0]))
    far = W[dw[W] == dw[W].max()]
    assert r2 == int(far.min())


@pytest.mark.parametrize("which", ["paper20", "rand4", "rand5", "grid"])
def test_every_edge_joins_equal_or_adjacent_sublevels(which):
    if which == "paper20":
        A = _golden_graph()
    elif which == "grid":
        A = w.stencil_3d27(5)
    else:
        A = _random_connected(80, 3, int(which[-1]), symmetric=False)
    d1, d2, perm, iperm = oracle.sublevels(A.n, A.rowptr, A.col, 0)
    for v in range(A.n):
        for e in range(A.rowptr[v], A.rowptr[v + 1]):
            u = A.col[e]
            assert abs(d1[u] - d1[v]) <= 1 and abs(d2[u] - d2[v]) <= 1, (v, u)
    # rows ordered by (level, sub-level, index): each level a run of sub-levels
    assert sorted(perm.tolist()) == list(range(A.n))
    keys = [(d1[v], d2[v], v) for v in perm]
    assert keys == sorted(keys)
    assert np.array_equal(iperm[perm], np.arange(A.n))


def test_paper_stencil_sublevels_split_its_bulky_levels():
    # the 20-vertex example of Fig. entire_stencil_figure: the sub-levels of
    # every level are graph distances from the second root, and the widest
    # level is split into more than one sub-level
    A = _golden_graph()
    d1, d2, _, _ = oracle.sublevels(A.n, A.rowptr, A.col, 0)
    M = sp.csr_matrix((np.ones(A.nnz), A.col, A.rowptr), shape=(A.n, A.n))
    r2 = oracle.sublevel_root(A.n, A.rowptr, A.col, 0)
    assert np.array_equal(d2, csg.shortest_path(M, unweighted=True, directed=False, indices=r2))
    widest = int(np.argmax(np.bincount(d1)))
    assert len(set(d2[d1 == widest].tolist())) > 1
