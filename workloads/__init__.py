"""Seeded synthetic inputs for the matrix power kernel.

This module builds the sparse matrices and dense vectors that both the
HIP path and the CPU oracle consume.  It contains no part of the method's
arithmetic (no products, no powers, no recurrences): only CSR assembly of
well-defined test matrices and seeded random draws.

Every matrix is returned as a :class:`CSR` with 0-based ``int32`` row
pointers and column indices and ``float64`` values; columns are stored in
ascending order within each row and there are no duplicate entries.

Row numbering of lattice matrices is ``i = x + L*(y + L*z)`` (x fastest).

Workloads (the paper's matrices are SuiteSparse/Lynx/ScaMaC files that are
not available here; these generators stand in for them with the same
shapes, row densities and structure):

* ``stencil_2d5(64)``       2D 5-point Laplacian, 64x64, truncated boundary.
* ``stencil_3d27(128)``     3D 27-point stencil, 128^3, truncated boundary.
* ``banded_random(2**22)``  symmetric-pattern random band, half-width 5000,
                            Poisson(15) off-diagonals per row, N(0,1) values,
                            symmetric permutation within 64k-row windows.
* ``anderson_3d(160)``      3D Anderson tight-binding Hamiltonian, periodic,
                            hopping -1, on-site U[-W/2, W/2] with W = 16.5,
                            scaled by 1/(W/2 + 6) into [-1, 1].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSR", "rng", "stencil_2d5", "stencil_3d27", "tridiag_1d", "banded_random",
    "anderson_3d", "identity", "permutation_matrix", "random_sparse",
    "from_dense", "uniform_vectors", "integer_vectors", "random_sign_unit_vectors",
    "random_phase_vectors", "config", "CONFIGS", "serving_pool_specs",
    "serving_requests", "build_pool_matrix",
]


@dataclasses.dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        if self.n > 4096:
            raise ValueError("to_dense is for tiny matrices only")
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        np.add.at(d, (rows, self.col), self.val)
        return d

    def check(self) -> None:
        assert self.rowptr.dtype == np.int32 and self.col.dtype == np.int32
        assert self.val.dtype == np.float64
        assert self.rowptr.shape == (self.n + 1,) and self.rowptr[0] == 0
        assert np.all(np.diff(self.rowptr) >= 0)
        assert self.col.shape == (self.nnz,) and self.val.shape == (self.nnz,)
        if self.nnz:
            assert self.col.min() >= 0 and self.col.max() < self.n


def rng(seed: int) -> np.random.Generator:
    """The one seeded generator used for every random draw here."""
    return np.random.Generator(np.random.PCG64(seed))


def _from_padded(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray, name: str) -> CSR:
    """Compress an (n, k) padded neighbour table into CSR (row-major order)."""
    n = cols.shape[0]
    counts = mask.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return CSR(n, rowptr.astype(np.int32), cols[mask].astype(np.int32, copy=False),
               vals[mask].astype(np.float64, copy=False), name)


def _lattice_stencil(dims: tuple, offsets: list, weights: list, periodic: bool,
                     name: str, diag_values: np.ndarray | None = None) -> CSR:
    """CSR of a stencil on a lattice with ``dims = (Lx, Ly, Lz)``.

    ``offsets`` are (dx, dy, dz) tuples, ``weights`` the matching coefficient
    (the (0,0,0) weight is replaced by ``diag_values`` when given).  With a
    truncated boundary, neighbours outside the box are dropped; with a
    periodic boundary they wrap.  Columns are sorted ascending per row.
    """
    Lx, Ly, Lz = dims
    n = Lx * Ly * Lz
    idx = np.arange(n, dtype=np.int64)
    x = idx % Lx
    y = (idx // Lx) % Ly
    z = idx // (Lx * Ly)
    k = len(offsets)
    cols = np.empty((n, k), dtype=np.int64)
    vals = np.empty((n, k), dtype=np.float64)
    mask = np.ones((n, k), dtype=bool)
    for j, ((dx, dy, dz), w) in enumerate(zip(offsets, weights)):
        xx, yy, zz = x + dx, y + dy, z + dz
        if periodic:
            xx %= Lx
            yy %= Ly
            zz %= Lz
        else:
            mask[:, j] = (xx >= 0) & (xx < Lx) & (yy >= 0) & (yy < Ly) & (zz >= 0) & (zz < Lz)
        cols[:, j] = xx + Lx * (yy + Ly * zz)
        if (dx, dy, dz) == (0, 0, 0) and diag_values is not None:
            vals[:, j] = diag_values
        else:
            vals[:, j] = w
    if periodic:
        # wrapped neighbours break the ascending order near the faces
        order = np.argsort(cols, axis=1, kind="stable")
        cols = np.take_along_axis(cols, order, axis=1)
        vals = np.take_along_axis(vals, order, axis=1)
        if np.any(cols[:, 1:] == cols[:, :-1]):
            raise ValueError("periodic lattice too small: duplicate neighbours")
    else:
        cols = np.where(mask, cols, 0)
    return _from_padded(cols, vals, mask, name)


def stencil_2d5(L: int, diag: float = 4.0, off: float = -1.0) -> CSR:
    """2D 5-point Laplacian on an L x L grid with truncated (Dirichlet) boundary."""
    offs = [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)]
    w = [off, off, diag, off, off]
    return _lattice_stencil((L, L, 1), offs, w, False, f"stencil2d5_{L}")


def stencil_3d27(L: int, diag: float = 26.0, off: float = -1.0) -> CSR:
    """3D 27-point stencil on an L^3 grid with truncated (Dirichlet) boundary."""
    offs, w = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                offs.append((dx, dy, dz))
                w.append(diag if (dx, dy, dz) == (0, 0, 0) else off)
    return _lattice_stencil((L, L, L), offs, w, False, f"stencil3d27_{L}")


def tridiag_1d(n: int, diag: float = 2.0, off: float = -1.0, periodic: bool = False) -> CSR:
    """1D three-point stencil tridiag(off, diag, off)."""
    offs = [(-1, 0, 0), (0, 0, 0), (1, 0, 0)]
    return _lattice_stencil((n, 1, 1), offs, [off, diag, off], periodic, f"tridiag_{n}")


def anderson_3d(L: int, seed: int = 2004, W: float = 16.5, t: float = 1.0,
                periodic: bool = True, scale: bool = True) -> CSR:
    """3D Anderson tight-binding Hamiltonian on an L^3 lattice.

    On-site energies (W/2) * w_r with w_r ~ U[-1, 1]; nearest-neighbour
    hopping -t.  With ``scale`` the matrix is divided by the Gershgorin
    bound W/2 + 6|t| so that its spectrum lies in [-1, 1].
    """
    n = L ** 3
    w = rng(seed).uniform(-1.0, 1.0, size=n)
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    wts = [-t] * 7
    A = _lattice_stencil((L, L, L), offs, wts, periodic, f"anderson_{L}",
                         diag_values=(W / 2.0) * w)
    if scale:
        A.val /= (W / 2.0 + 6.0 * abs(t))
    return A


def identity(n: int) -> CSR:
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
               np.ones(n), f"identity_{n}")


def permutation_matrix(n: int, seed: int) -> tuple[CSR, np.ndarray]:
    """P with P[i, sigma[i]] = 1, so (P x)[i] = x[sigma[i]].  Returns (P, sigma)."""
    sigma = rng(seed).permutation(n).astype(np.int32)
    return CSR(n, np.arange(n + 1, dtype=np.int32), sigma.copy(), np.ones(n),
               f"perm_{n}"), sigma


def from_dense(d: np.ndarray, name: str = "dense") -> CSR:
    n = d.shape[0]
    mask = d != 0
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(counts)
    rows, cols = np.nonzero(mask)
    return CSR(n, rowptr, cols.astype(np.int32), d[rows, cols].astype(np.float64), name)


def random_sparse(n: int, density: float, seed: int, symmetric_pattern: bool = False,
                  diag: bool = True, values: str = "normal") -> CSR:
    """Small unstructured test matrix (non-symmetric values)."""
    g = rng(seed)
    m = g.random((n, n)) < density
    if symmetric_pattern:
        m = m | m.T
    if diag:
        np.fill_diagonal(m, True)
    if values == "normal":
        v = g.standard_normal((n, n))
    elif values == "int":
        v = g.integers(-2, 3, size=(n, n)).astype(np.float64)
        v[v == 0] = 1.0
    else:
        raise ValueError(values)
    return from_dense(np.where(m, v, 0.0), f"rand_{n}")


def banded_random(n: int = 2 ** 22, half_width: int = 5000, mean_offdiag: float = 15.0,
                  seed: int = 2003, window: int = 65536, perm_seed: int = 3003,
                  permute: bool = True) -> CSR:
    """Irregular banded random matrix with a symmetric pattern.

    Row i draws Poisson(mean_offdiag/2) offsets uniform in [1, half_width]
    above the diagonal; the pattern is mirrored (so each row has about
    Poisson(mean_offdiag) off-diagonal entries), the diagonal is added and
    duplicates are merged.  Values are i.i.d. N(0,1) per stored entry (the
    values are not symmetric).  Finally a symmetric permutation P A P^T
    shuffles rows and columns within consecutive windows of ``window`` rows.
    """
    g = rng(seed)
    cnt = g.poisson(mean_offdiag / 2.0, size=n)
    src = np.repeat(np.arange(n, dtype=np.int64), cnt)
    dst = src + g.integers(1, half_width + 1, size=src.size)
    keep = dst < n
    src, dst = src[keep], dst[keep]
    diag = np.arange(n, dtype=np.int64)
    key = np.concatenate([src * n + dst, dst * n + src, diag * n + diag])
    del src, dst
    key = np.unique(key)  # sorted, duplicates merged
    rows = key // n
    cols = key - rows * n
    del key
    vals = g.standard_normal(rows.size)
    if permute:
        pg = rng(perm_seed)
        perm = np.arange(n, dtype=np.int64)  # new index -> old index
        for s in range(0, n, window):
            e = min(n, s + window)
            perm[s:e] = s + pg.permutation(e - s)
        iperm = np.empty(n, dtype=np.int64)
        iperm[perm] = np.arange(n, dtype=np.int64)
        rows = iperm[rows]
        cols = iperm[cols]
        order = np.argsort(rows * n + cols, kind="stable")
        rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32")
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64),
               f"banded_{n}")


# ---------------------------------------------------------------- vectors

def uniform_vectors(n: int, R: int, seed: int) -> np.ndarray:
    """x uniform in [-1, 1), shape (n, R), row-major (RHS fastest)."""
    return rng(seed).uniform(-1.0, 1.0, size=(n, R))


def integer_vectors(n: int, R: int, seed: int) -> np.ndarray:
    """x with entries in {-1, 0, 1}: stencil powers stay exact integers."""
    return rng(seed).integers(-1, 2, size=(n, R)).astype(np.float64)


def random_sign_unit_vectors(n: int, R: int, seed: int) -> np.ndarray:
    """Entries +-1/sqrt(n) with independent random signs (unit 2-norm columns)."""
    s = rng(seed).integers(0, 2, size=(n, R)).astype(np.float64) * 2.0 - 1.0
    return s / math.sqrt(n)


def random_phase_vectors(n: int, R: int, seed: int) -> np.ndarray:
    """Real stand-in for random-phase unit vectors: random signs, norm 1."""
    return random_sign_unit_vectors(n, R, seed)


# ---------------------------------------------------------------- configs

CONFIGS = {
    "stencil2d5_64_p4": dict(matrix=("stencil_2d5", 64), p=4, R=1, x=("uniform", 1001),
                             kind="powers"),
    "stencil3d27_128_p8": dict(matrix=("stencil_3d27", 128), p=8, R=1, x=("uniform", 1002),
                               kind="powers"),
    "banded_4m_p6": dict(matrix=("banded_random", 2 ** 22), p=6, R=1, x=("uniform", 1003),
                         kind="powers"),
    "anderson160_cheb16_r8": dict(matrix=("anderson_3d", 160), p=16, R=8,
                                  x=("sign_unit", 1004), kind="chebyshev"),
    # a block of 16 right-hand sides on a mid-size stencil: vector traffic
    # dominates and the blocking window fits the cache
    "stencil3d27_64_p16_r16": dict(matrix=("stencil_3d27", 64), p=16, R=16, x=("uniform", 1006),
                                   kind="powers"),
}


def _matrix(spec) -> CSR:
    kind, size = spec
    if kind == "stencil_2d5":
        return stencil_2d5(size)
    if kind == "stencil_3d27":
        return stencil_3d27(size)
    if kind == "banded_random":
        return banded_random(size)
    if kind == "anderson_3d":
        return anderson_3d(size)
    raise ValueError(kind)


def _vectors(spec, n: int, R: int) -> np.ndarray:
    kind, seed = spec
    if kind == "uniform":
        return uniform_vectors(n, R, seed)
    if kind == "integer":
        return integer_vectors(n, R, seed)
    if kind == "sign_unit":
        return random_sign_unit_vectors(n, R, seed)
    raise ValueError(kind)


def config(name: str):
    """Return (A, x, p, kind) for a named workload."""
    c = CONFIGS[name]
    A = _matrix(c["matrix"])
    x = _vectors(c["x"], A.n, c["R"])
    return A, x, c["p"], c["kind"]


# ---------------------------------------------------------------- serving stream

def serving_pool_specs():
    """The six device-resident matrices of the serving stream (N from 1e4 to 4.1e6)."""
    return [("stencil_2d5", 100), ("stencil_2d5", 1000), ("stencil_3d27", 64),
            ("stencil_3d27", 128), ("anderson_3d", 50), ("anderson_3d", 160)]


def build_pool_matrix(spec) -> CSR:
    kind, size = spec
    if kind == "anderson_3d":
        return anderson_3d(size, seed=2004 + size)
    return _matrix(spec)


def serving_requests(n_requests: int = 512, rate_per_s: float = 1000.0, seed: int = 5005,
                     pool_size: int = 6, p_range=(4, 32), rhs_choices=(1, 2, 4, 8, 16)):
    """Poisson arrivals; each request draws (matrix id, p, R, x seed).

    Returns a list of dicts sorted by arrival time (seconds from start).
    """
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    mats = g.integers(0, pool_size, size=n_requests)
    ps = g.integers(p_range[0], p_range[1] + 1, size=n_requests)
    rs = g.choice(np.asarray(rhs_choices), size=n_requests)
    xseeds = g.integers(0, 2 ** 31 - 1, size=n_requests)
    return [dict(id=i, t=float(t[i]), matrix=int(mats[i]), p=int(ps[i]), R=int(rs[i]),
                 x_seed=int(xseeds[i])) for i in range(n_requests)]
