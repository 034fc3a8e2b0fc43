"""CPU oracle for the level-blocked matrix power kernel.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does, and this package imports nothing from the product package.

Contents (each function names the passage of Lacey et al., "Cache Blocking of
Distributed-Memory Parallel Matrix Power Kernels", that it follows):

* :func:`powers`  -- y_k = A^k x, k = 1..p, as p back-to-back FP64 SpMVs
  (Sec. "RACE Applied to the Matrix Power Kernel"; Alg. 1 without halo
  exchange).  Implemented in plain C (``mpk_oracle.c``), sequential in-row
  accumulation, no fused multiply-add.
* :func:`recur`   -- the three-term recurrence of the Chebyshev application,
  Eq. (anderson_spmv), with general coefficients.
* :func:`poly_sums` -- weighted sums sum_k w_k y_k of the recurrence's
  vectors, the polynomial that one Chebyshev time step evaluates
  (Sec. "Application: Chebyshev Time Propagation", the expansion of
  exp(-i dt H) in J_k(dt) and the vectors v_k).
* :func:`cheb_time_coefficients` / :func:`cheb_time_step` -- that expansion
  written out: c_0 = J_0(dt), c_k = 2 (-i)^k J_k(dt), applied to a complex
  state stored as pairs of real columns.
* :func:`bfs_levels` -- the level sets of Sec. "RACE Applied to the Matrix
  Power Kernel" (the case equation for L(i)), computed literally with set
  operations on the symmetrised graph G(A).
* :func:`pseudo_peripheral_root` -- a BFS root far from the rest of the
  graph (the root choice the paper leaves open when it roots the levels at
  row 0), by the George-Liu iteration.
* :func:`lp_diagonal_order` -- the LB-MPK traversal of the Lp diagram: the
  diagonals i + p = const in increasing order, each walked from bottom-right
  (largest level) to top-left (Fig. lp_basic).
* :func:`sublevel_root` / :func:`sublevels` -- levels broken into
  sub-levels (the paper's recursion stage s_m, Sec. "Experimental Setup",
  breaks bulky levels down; it gives no construction, so this is a
  reading): a second breadth-first distance d2 from a second root is taken
  over the whole graph, and the sub-level of a vertex is the pair (its level,
  d2).  Both coordinates change by at most one along any edge, so every edge
  joins equal or adjacent sub-levels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpk_oracle.c")
_LIB = os.path.join(_HERE, "libmpk_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, -O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_powers.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int, P,
                                      ctypes.c_int, P, ctypes.c_int]
        lib.oracle_powers.restype = ctypes.c_int
        lib.oracle_recur.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int, ctypes.c_int, P,
                                     ctypes.c_int, P, P, P, P, ctypes.c_int]
        lib.oracle_recur.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _prep(A, x, value_bits):
    rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    if value_bits == 32:
        val = np.ascontiguousarray(A.val, dtype=np.float32)
    elif value_bits == 64:
        val = np.ascontiguousarray(A.val, dtype=np.float64)
    else:
        raise ValueError("value_bits must be 32 or 64")
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    if x.shape[0] != A.n:
        raise ValueError("x has the wrong number of rows")
    return rowptr, col, val, x


def threads() -> int:
    return int(_load().oracle_threads())


def powers(A, x: np.ndarray, p: int, value_bits: int = 64, nthreads: int = 0) -> np.ndarray:
    """All powers y_k = A^k x, k = 1..p; returns Y of shape (p, n, R).

    Each y_k is one SpMV of y_{k-1} (MPK definition, Sec. "RACE Applied to the
    Matrix Power Kernel"; the SpMV loop of Alg. 1).  ``value_bits=32`` rounds
    the stored values to float and promotes them before each product (the
    FP32-storage reading: vectors and sums stay FP64).
    """
    rowptr, col, val, x = _prep(A, x, value_bits)
    R = x.shape[1]
    Y = np.empty((p, A.n, R), dtype=np.float64)
    rc = _load().oracle_powers(A.n, _ptr(rowptr), _ptr(col), _ptr(val), value_bits, R, _ptr(x),
                               p, _ptr(Y), nthreads)
    if rc:
        raise ValueError(f"oracle_powers failed ({rc})")
    return Y


def recur(A, x: np.ndarray, alpha, beta, gamma, value_bits: int = 64,
          nthreads: int = 0) -> np.ndarray:
    """Three-term recurrence y_{j+1} = alpha_j A y_j + beta_j y_j + gamma_j y_{j-1}.

    j = 0..p-1 with y_0 = x and no gamma term at j = 0; returns (p, n, R).
    A coefficient that is exactly zero omits its term (the Chebyshev form has
    no beta term at all).
    The Chebyshev recurrence of Eq. (anderson_spmv) is alpha = (1, 2, 2, ...),
    beta = 0, gamma = (0, -1, -1, ...).
    """
    rowptr, col, val, x = _prep(A, x, value_bits)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    p = alpha.size
    if beta.size != p or gamma.size != p or p < 1:
        raise ValueError("coefficient arrays must have the same length p >= 1")
    R = x.shape[1]
    Y = np.empty((p, A.n, R), dtype=np.float64)
    rc = _load().oracle_recur(A.n, _ptr(rowptr), _ptr(col), _ptr(val), value_bits, R, _ptr(x),
                              p, _ptr(alpha), _ptr(beta), _ptr(gamma), _ptr(Y), nthreads)
    if rc:
        raise ValueError(f"oracle_recur failed ({rc})")
    return Y


def chebyshev_coefficients(p: int):
    """alpha, beta, gamma of the Chebyshev recurrence (v_1 = H v_0, then 2H v_k - v_{k-1})."""
    alpha = np.full(p, 2.0)
    alpha[0] = 1.0
    beta = np.zeros(p)
    gamma = np.full(p, -1.0)
    gamma[0] = 0.0
    return alpha, beta, gamma


def poly_sums(A, x: np.ndarray, alpha, beta, gamma, wa, wb=None, value_bits: int = 64,
              nthreads: int = 0):
    """Weighted sums acc = sum_{k=0..p} w[k] y_k of the recurrence's vectors.

    y_0 = x and y_1..y_p come from :func:`recur` (p = len(alpha)); wa and wb
    hold p + 1 weights each.  The sum runs in increasing k: its first term
    with a nonzero weight is w[k]*y_k, every later one is added as
    acc + w[k]*y_k; a weight that is exactly zero omits its term, and a sum
    whose weights are all zero is the zero vector.  This is the polynomial
    evaluation of one Chebyshev time step (Sec. "Application: Chebyshev Time
    Propagation").  Returns (acc_a, acc_b), each (n, R); acc_b is None when
    wb is None.
    """
    rowptr, col, val, x = _prep(A, x, value_bits)
    Y = recur(A, x, alpha, beta, gamma, value_bits=value_bits, nthreads=nthreads)
    p = Y.shape[0]

    def one(w):
        w = np.asarray(w, dtype=np.float64)
        if w.shape != (p + 1,):
            raise ValueError("weights must hold p + 1 values")
        acc = None
        for k in range(p + 1):
            if w[k] == 0.0:
                continue
            t = w[k] * (x if k == 0 else Y[k - 1])
            acc = t if acc is None else acc + t
        return np.zeros_like(x) if acc is None else acc

    return one(wa), (None if wb is None else one(wb))


def cheb_time_coefficients(M: int, dt: float):
    """Chebyshev expansion of exp(-i dt H) kept to M + 1 terms.

    Sec. "Application: Chebyshev Time Propagation": the step is
    J_0(dt) v_0 + 2 sum_{k=1..M} (-i)^k J_k(dt) v_k with v_0 = psi,
    v_1 = H psi and v_{k+1} = 2 H v_k - v_{k-1} (valid for a spectrum inside
    [-1, 1]).  Returns (alpha, beta, gamma) of that recurrence (M powers) and
    (wa, wb), the real and imaginary parts of the M + 1 expansion weights.
    (-i)^k cycles through 1, -i, -1, i, so every weight is purely real (k
    even) or purely imaginary (k odd), with the other part exactly zero.
    """
    from scipy.special import jv
    if M < 1:
        raise ValueError("M must be at least 1")
    J = jv(np.arange(M + 1), float(dt))
    wa = np.zeros(M + 1)
    wb = np.zeros(M + 1)
    wa[0] = J[0]
    for k in range(1, M + 1):
        re, im = ((1.0, 0.0), (0.0, -1.0), (-1.0, 0.0), (0.0, 1.0))[k % 4]
        if re:
            wa[k] = 2.0 * re * J[k]
        if im:
            wb[k] = 2.0 * im * J[k]
    alpha, beta, gamma = chebyshev_coefficients(M)
    return alpha, beta, gamma, wa, wb


def combine_complex(acc_a: np.ndarray, acc_b: np.ndarray) -> np.ndarray:
    """Complex result of the two real weighted sums, on column pairs.

    With column 2j the real and 2j+1 the imaginary part of state j and
    complex weights c_k = wa_k + i wb_k, sum_k c_k v_k has real part
    acc_a[:, 2j] - acc_b[:, 2j+1] and imaginary part
    acc_a[:, 2j+1] + acc_b[:, 2j] (H is real, so it acts on each part alone).
    """
    out = np.empty_like(acc_a)
    out[:, 0::2] = acc_a[:, 0::2] - acc_b[:, 1::2]
    out[:, 1::2] = acc_a[:, 1::2] + acc_b[:, 0::2]
    return out


def cheb_time_step(A, psi: np.ndarray, dt: float, M: int, value_bits: int = 64,
                   nthreads: int = 0) -> np.ndarray:
    """One Chebyshev time step psi -> exp(-i dt H) psi (truncated after M).

    psi is real (n, 2m): column 2j holds the real and 2j+1 the imaginary part
    of state j.  Returns the stepped states in the same layout.
    """
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    if psi.ndim != 2 or psi.shape[1] % 2:
        raise ValueError("psi must be (n, 2m): real and imaginary columns")
    al, be, ga, wa, wb = cheb_time_coefficients(M, dt)
    acc_a, acc_b = poly_sums(A, psi, al, be, ga, wa, wb, value_bits=value_bits,
                             nthreads=nthreads)
    return combine_complex(acc_a, acc_b)


# ------------------------------------------------------------ graph side

def neighbour_sets(n: int, rowptr, col):
    """N(u) on G(A): an edge joins v and j for every stored entry (v, j).

    Values play no role, self-loops are dropped and the pattern is taken as
    symmetric (the paper's note on non-symmetric matrices: missing mirror
    entries are filled in for the level construction only).
    """
    N = [set() for _ in range(n)]
    for v in range(n):
        for e in range(int(rowptr[v]), int(rowptr[v + 1])):
            j = int(col[e])
            if j != v:
                N[v].add(j)
                N[j].add(v)
    return N


def bfs_levels(n: int, rowptr, col, root: int = 0):
    """Level sets L(0), L(1), ... of G(A) by the paper's case equation.

    L(0) = {root}; L(1) = N(L(0)); L(i) = N(L(i-1)) minus N(L(i-2)) minus
    L(i-2) for i >= 2.  When a level comes out empty while vertices remain
    (a disconnected graph), the next level restarts at the lowest unvisited
    vertex.  Inside a level, vertices are listed in ascending original index.
    Returns (levels, perm, iperm) with perm[new] = old and iperm[old] = new.
    """
    N = neighbour_sets(n, rowptr, col)

    def nb(S):
        out = set()
        for u in S:
            out |= N[u]
        return out

    levels = []
    seen = set()
    if n and not 0 <= root < n:
        raise ValueError("root out of range")
    if n == 0:
        return levels, np.zeros(0, np.int64), np.zeros(0, np.int64)
    prev2, prev1 = None, None
    while len(seen) < n:
        if prev1 is None:
            start = root if not levels else min(set(range(n)) - seen)
            cur = {start}
        elif prev2 is None:
            cur = nb(prev1) - prev1
        else:
            cur = nb(prev1) - nb(prev2) - prev2
        # the case equation never yields an already-levelled vertex
        assert not (cur & seen), "level equation revisited a vertex"
        if not cur:
            prev2, prev1 = None, None
            continue
        levels.append(sorted(cur))
        seen |= cur
        prev2, prev1 = prev1, cur
    perm = np.array([v for L in levels for v in L], dtype=np.int64)
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    return levels, perm, iperm


def pseudo_peripheral_root(n: int, rowptr, col, start: int = 0) -> int:
    """A pseudo-peripheral vertex of start's component of G(A) (George-Liu).

    Take x = start.  Repeatedly run a breadth-first search from x and pick,
    in its last distance layer, the vertex y of smallest degree (number of
    distinct neighbours other than itself; ties to the smaller index).  If
    y's eccentricity exceeds x's, continue from y; otherwise x is the
    result.  The levels of the paper rooted at this vertex are as many and
    as thin as this heuristic can make them.
    """
    if n == 0:
        return 0
    N = neighbour_sets(n, rowptr, col)

    def layers(r):
        dist = {r: 0}
        front = [r]
        out = [front]
        while True:
            nxt = sorted({v for u in front for v in N[u] if v not in dist})
            if not nxt:
                return out
            for v in nxt:
                dist[v] = len(out)
            out.append(nxt)
            front = nxt

    x = start
    Lx = layers(x)
    while True:
        last = Lx[-1]
        y = min(last, key=lambda v: (len(N[v]), v))
        Ly = layers(y)
        if len(Ly) > len(Lx):
            x, Lx = y, Ly
        else:
            return x


def lp_diagonal_order(n_levels: int, p_m: int):
    """Execution order of the Lp diagram (Fig. lp_basic).

    The diagonals i + p = const are taken for const = 1, 2, ...; on each,
    cells go from the largest level (bottom-right, p small) to the smallest
    level (top-left, p large).  Returns the list of (level, power).
    """
    order = []
    for const in range(1, n_levels + p_m):
        for i in range(n_levels - 1, -1, -1):
            p = const - i
            if 1 <= p <= p_m:
                order.append((i, p))
    return order


def permute_csr(A, perm):
    """Symmetric permutation P A P^T with perm[new] = old, in-row order kept (Sec.
    "RACE Applied to the Matrix Power Kernel", BFS reordering)."""
    n = A.n
    iperm = np.empty(n, dtype=np.int64)
    iperm[np.asarray(perm)] = np.arange(n)
    counts = np.diff(A.rowptr.astype(np.int64))[perm]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = np.empty(A.nnz, dtype=np.int32)
    val = np.empty(A.nnz, dtype=np.float64)
    for new in range(n):
        old = int(perm[new])
        s, e = int(A.rowptr[old]), int(A.rowptr[old + 1])
        col[rowptr[new]:rowptr[new + 1]] = iperm[A.col[s:e]]
        val[rowptr[new]:rowptr[new + 1]] = A.val[s:e]
    return type(A)(n, rowptr.astype(np.int32), col, val, A.name + "_perm")


def _distances(n: int, rowptr, col, root: int):
    """d(v) = index of v's level in bfs_levels(root): the graph distance from
    root inside root's component; later components continue the count."""
    levels, _, _ = bfs_levels(n, rowptr, col, root)
    d = np.empty(n, dtype=np.int64)
    for i, L in enumerate(levels):
        d[np.asarray(L, dtype=np.int64)] = i
    return d


def sublevel_root(n: int, rowptr, col, root: int = 0) -> int:
    """Second root for the sub-levels of the levels rooted at `root`.

    Reading (the paper gives none): take the widest level W of
    bfs_levels(root) (the first one among equals), its smallest vertex w, and
    return the vertex of W farthest from w in G(A) (ties to the smaller
    index).  On a grid this puts the second root at the other end of the
    widest level, so that the second distance runs across the levels.
    """
    if n == 0:
        return 0
    levels, _, _ = bfs_levels(n, rowptr, col, root)
    W = max(levels, key=len)  # max returns the first widest
    w = W[0]
    d = _distances(n, rowptr, col, w)
    return max(W, key=lambda v: (d[v], -v))


def sublevels(n: int, rowptr, col, root: int = 0, root2=None):
    """Sub-levels of the levels rooted at `root`.

    d1(v) is v's level in bfs_levels(root), d2(v) its level in
    bfs_levels(root2) (root2 = sublevel_root(root) when None).  Rows are
    ordered by (d1, d2, original index): each level is a run of sub-levels.
    Returns (d1, d2, perm, iperm) with perm[new] = old.
    """
    if root2 is None:
        root2 = sublevel_root(n, rowptr, col, root)
    d1 = _distances(n, rowptr, col, root)
    d2 = _distances(n, rowptr, col, root2)
    perm = np.array(sorted(range(n), key=lambda v: (d1[v], d2[v], v)), dtype=np.int64)
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n)
    return d1, d2, perm, iperm
