"""Seeded synthetic workloads for block-multicolored ICCG.

This module only draws random numbers and assembles sparse SPD matrices,
right-hand sides and probe vectors.  It holds none of the solver's arithmetic
(no ordering, no factorization, no substitution, no Krylov step), so both the
CPU oracle and the GPU library can be fed from it without sharing any method
code.

The paper evaluates on eight SuiteSparse SPD matrices (Section 5, Table 1)
which are not available here.  The generators below are synthetic stand-ins
with the same structure classes:

* a 2D 5-point Laplacian (small latency-bound case),
* a 3D 7-point variable-coefficient Poisson operator (ANZR about 7, like
  parabolic_fem / ecology2 / thermal2),
* an FEM-like symmetric k-nearest-neighbour graph Laplacian on random points
  (unstructured, like apache2 / G3_circuit),
* a 3D 27-point operator (high ANZR, like Emilia_923 / Geo_1438 / Hook_1498).

All matrices are returned as CSR with int32 indices, sorted column indices and
the diagonal stored, which is the input format of both sides.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "grid2d_5pt", "grid3d_7pt_lognormal", "grid3d_27pt_lognormal",
    "knn_laplacian", "uniform_rhs", "gaussian_probes", "workload",
    "path_graph_matrix", "random_spd_mmatrix", "WORKLOADS",
]


@dataclass
class CSR:
    """Square sparse matrix in compressed sparse row form (int32 indices)."""
    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray     # int32[nnz], ascending inside each row
    val: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        out = np.zeros((self.n, self.n))
        for i in range(self.n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                out[i, self.col[k]] += self.val[k]
        return out


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Assemble CSR from COO triplets (no duplicate (row, col) pairs expected)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], np.asarray(vals, dtype=np.float64)[order]
    if rows.size > 1:
        dup = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if dup.any():
            raise ValueError("duplicate entries in COO assembly")
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals)


def _edge_matrix(n: int, lo: np.ndarray, hi: np.ndarray, w: np.ndarray, shift: float) -> CSR:
    """Weighted graph Laplacian plus shift: a_ij = -w_ij, a_ii = sum_j w_ij + shift.

    The diagonal is accumulated in the fixed order of the edge list (np.add.at
    is unbuffered and sequential), so it is reproducible bit for bit.
    """
    diag = np.full(n, 0.0)
    np.add.at(diag, lo, w)
    np.add.at(diag, hi, w)
    diag += shift
    ar = np.arange(n, dtype=np.int64)
    rows = np.concatenate([lo, hi, ar])
    cols = np.concatenate([hi, lo, ar])
    vals = np.concatenate([-w, -w, diag])
    return _from_coo(n, rows, cols, vals)


def grid2d_5pt(nx: int, ny: int) -> CSR:
    """2D 5-point Laplacian, Dirichlet: a_ii = 4, a_ij = -1 to in-grid neighbours.

    Index i = x + nx*y.
    """
    n = nx * ny
    idx = np.arange(n, dtype=np.int64).reshape(ny, nx)
    lo_x, hi_x = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    lo_y, hi_y = idx[:-1, :].ravel(), idx[1:, :].ravel()
    lo = np.concatenate([lo_x, lo_y])
    hi = np.concatenate([hi_x, hi_y])
    ar = np.arange(n, dtype=np.int64)
    rows = np.concatenate([lo, hi, ar])
    cols = np.concatenate([hi, lo, ar])
    vals = np.concatenate([-np.ones(lo.size), -np.ones(lo.size), np.full(n, 4.0)])
    return _from_coo(n, rows, cols, vals)


def _faces_3d(nx: int, ny: int, nz: int):
    """Interior faces of an nx*ny*nz cell grid: x-faces, then y, then z.

    Within each direction the faces are in ascending order of the lower cell
    index i = x + nx*(y + ny*z).
    """
    idx = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    pairs = [
        (idx[:, :, :-1].ravel(), idx[:, :, 1:].ravel()),
        (idx[:, :-1, :].ravel(), idx[:, 1:, :].ravel()),
        (idx[:-1, :, :].ravel(), idx[1:, :, :].ravel()),
    ]
    return pairs


def grid3d_7pt_lognormal(nx: int, ny: int, nz: int, sigma: float, shift: float,
                         rng: np.random.Generator) -> CSR:
    """3D 7-point variable-coefficient Poisson operator.

    One coefficient c = exp(sigma * N(0,1)) per interior face, drawn for the
    x-faces, then the y-faces, then the z-faces, each in ascending lower-cell
    order.  a_ij = -c, a_ii = sum of the cell's face coefficients + shift
    (interior faces only, so shift alone keeps the operator nonsingular).
    """
    n = nx * ny * nz
    los, his, ws = [], [], []
    for lo, hi in _faces_3d(nx, ny, nz):
        los.append(lo)
        his.append(hi)
        ws.append(np.exp(sigma * rng.standard_normal(lo.size)))
    return _edge_matrix(n, np.concatenate(los), np.concatenate(his), np.concatenate(ws), shift)


def _offsets_27():
    """The 13 neighbour offsets (dx, dy, dz) with positive linear offset, ascending."""
    out = []
    for dz in (0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dz == 0 and (dy < 0 or (dy == 0 and dx <= 0)):
                    continue
                out.append((dx, dy, dz))
    return out


def grid3d_27pt_lognormal(m: int, sigma: float, shift: float, rng: np.random.Generator) -> CSR:
    """3D 27-point operator on an m^3 grid.

    One coefficient c = exp(sigma * N(0,1)) per undirected neighbour pair,
    drawn offset by offset (the 13 positive offsets in ascending linear order),
    each in ascending lower-cell order.  a_ij = -c, a_ii = sum + shift.
    """
    n = m ** 3
    z, y, x = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    lin = np.arange(n, dtype=np.int64)
    los, his, ws = [], [], []
    for dx, dy, dz in _offsets_27():
        ok = (x + dx >= 0) & (x + dx < m) & (y + dy >= 0) & (y + dy < m) & (z + dz < m)
        lo = lin[ok]
        hi = lo + dx + m * (dy + m * dz)
        los.append(lo)
        his.append(hi)
        ws.append(np.exp(sigma * rng.standard_normal(lo.size)))
    return _edge_matrix(n, np.concatenate(los), np.concatenate(his), np.concatenate(ws), shift)


def _morton10(p: np.ndarray) -> np.ndarray:
    """30-bit Morton code of the 10-bit cell coordinates of points in [0,1)^3."""
    cell = np.minimum((p * 1024.0).astype(np.int64), 1023)
    code = np.zeros(p.shape[0], dtype=np.int64)
    for bit in range(10):
        for d in range(3):
            code |= ((cell[:, d] >> bit) & 1) << (3 * bit + d)
    return code


def knn_laplacian(npts: int, k: int, shift: float, rng: np.random.Generator,
                  morton: bool = True) -> CSR:
    """FEM-like unstructured SPD matrix from a symmetric k-NN graph.

    Points are drawn U[0,1)^3, optionally sorted by the Morton code of their
    10-bit cell (an application-like numbering), then each point is joined to
    its k nearest other points; the union of both directions is kept.
    a_ij = -1/|p_i - p_j|, a_ii = sum_j 1/|p_i - p_j| + shift.
    """
    from scipy.spatial import cKDTree

    pts = rng.random((npts, 3))
    if morton:
        pts = pts[np.argsort(_morton10(pts), kind="stable")]
    tree = cKDTree(pts)
    _, nb = tree.query(pts, k=k + 1, workers=-1)
    nb = np.asarray(nb, dtype=np.int64)
    rows = np.repeat(np.arange(npts, dtype=np.int64), k + 1)
    cols = nb.ravel()
    keep = rows != cols
    rows, cols = rows[keep], cols[keep]
    # at most k neighbours per point (drop the (k+1)-th if self was not among the k+1)
    cnt = np.bincount(rows, minlength=npts)
    first = np.zeros(npts + 1, dtype=np.int64)
    np.cumsum(cnt, out=first[1:])
    pos = np.arange(rows.size) - first[rows]
    keep = pos < k
    rows, cols = rows[keep], cols[keep]
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    key = np.unique(lo * npts + hi)
    lo, hi = key // npts, key % npts
    w = 1.0 / np.linalg.norm(pts[lo] - pts[hi], axis=1)
    return _edge_matrix(npts, lo, hi, w, shift)


def path_graph_matrix(n: int) -> CSR:
    """1D Laplacian tridiag(-1, 2, -1) in natural order."""
    lo = np.arange(n - 1, dtype=np.int64)
    ar = np.arange(n, dtype=np.int64)
    rows = np.concatenate([lo, lo + 1, ar])
    cols = np.concatenate([lo + 1, lo, ar])
    vals = np.concatenate([-np.ones(n - 1), -np.ones(n - 1), np.full(n, 2.0)])
    return _from_coo(n, rows, cols, vals)


def random_spd_mmatrix(n: int, density: float, rng: np.random.Generator,
                       shift: float = 0.1) -> CSR:
    """Random symmetric diagonally dominant M-matrix (IC(0) never breaks down)."""
    mask = np.triu(rng.random((n, n)) < density, 1)
    lo, hi = np.nonzero(mask)
    w = rng.uniform(0.1, 2.0, lo.size)
    return _edge_matrix(n, lo.astype(np.int64), hi.astype(np.int64), w, shift)


def uniform_rhs(n: int, rng: np.random.Generator) -> np.ndarray:
    """b = 2u - 1, u ~ U[0,1)."""
    return 2.0 * rng.random(n) - 1.0


def gaussian_probes(n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """count probe vectors z ~ N(0, I), shape [count, n]."""
    return rng.standard_normal((count, n))


# Named workloads.  Each returns (A, b) with the matrix draws first and the
# right-hand side drawn afterwards from the same generator.
def _w_grid2d(seed):
    rng = np.random.default_rng(seed)
    A = grid2d_5pt(64, 64)
    return A, uniform_rhs(A.n, rng)


def _w_poisson7(m):
    def make(seed):
        rng = np.random.default_rng(seed)
        A = grid3d_7pt_lognormal(m, m, m, 1.0, 1e-6, rng)
        return A, uniform_rhs(A.n, rng)
    return make


def _w_knn(npts):
    def make(seed):
        rng = np.random.default_rng(seed)
        A = knn_laplacian(npts, 13, 1e-3, rng)
        return A, uniform_rhs(A.n, rng)
    return make


def _w_stencil27(m):
    def make(seed):
        rng = np.random.default_rng(seed)
        A = grid3d_27pt_lognormal(m, 2.0, 1e-6, rng)
        return A, uniform_rhs(A.n, rng)
    return make


def _w_randspd(n, density):
    def make(seed):
        rng = np.random.default_rng(seed)
        A = random_spd_mmatrix(n, density, rng)
        return A, uniform_rhs(A.n, rng)
    return make


def _w_learned(m):
    def make(seed):
        rng = np.random.default_rng(seed)
        sigma = rng.uniform(0.5, 2.0)
        A = grid3d_7pt_lognormal(m, m, m, sigma, 1e-6, rng)
        return A, uniform_rhs(A.n, rng)
    return make


WORKLOADS = {
    "laplace2d_64": _w_grid2d,            # n=4,096
    "poisson7_128": _w_poisson7(128),     # n=2,097,152
    "poisson7_64": _w_poisson7(64),
    "poisson7_32": _w_poisson7(32),
    "poisson7_16": _w_poisson7(16),
    "knn13_1m": _w_knn(1_000_000),
    "knn13_100k": _w_knn(100_000),
    "knn13_20k": _w_knn(20_000),
    "stencil27_96": _w_stencil27(96),     # n=884,736
    "stencil27_32": _w_stencil27(32),
    "stencil27_12": _w_stencil27(12),
    "randspd_2k": _w_randspd(2000, 0.03),  # about 60 neighbours per row
    "randspd6_2k": _w_randspd(2000, 0.003),  # about 6 neighbours per row (rows of 9-16 entries after ordering)
    "lognormal7_32": _w_learned(32),      # learned-form training matrices
    "lognormal7_64": _w_learned(64),
    "lognormal7_128": _w_learned(128),
}


def workload(name: str, seed: int = 42):
    """(A, b) for a named synthetic workload."""
    return WORKLOADS[name](seed)


def from_edges(n: int, edges, shift: float = 1.0, weight: float = 1.0) -> CSR:
    """Graph Laplacian (unit weights) plus shift for an explicit undirected edge list."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    return _edge_matrix(n, lo, hi, np.full(lo.size, float(weight)), shift)


def clique_ring(k: int, m: int, ring: bool = True) -> CSR:
    """k cliques of m nodes; consecutive cliques joined by one edge (a ring if ring)."""
    edges = []
    for c in range(k):
        base = c * m
        edges += [(base + a, base + b) for a in range(m) for b in range(a + 1, m)]
    links = k if ring else k - 1
    for c in range(links):
        edges.append((c * m + m - 1, ((c + 1) % k) * m))
    return from_edges(k * m, edges)


def banded_graph(n: int, width: int) -> CSR:
    """Nodes 0..n-1 with edges i~i+1 (same row of length width) and i~i+width."""
    i = np.arange(n, dtype=np.int64)
    a = i[(i % width != width - 1) & (i + 1 < n)]
    b = i[i + width < n]
    lo = np.concatenate([a, b])
    hi = np.concatenate([a + 1, b + width])
    return _edge_matrix(n, lo, hi, np.ones(lo.size), 1.0)


def glorot_params(shapes, seed: int, zero=("b", "bm", "br", "wo", "bo")) -> np.ndarray:
    """Concatenated parameter vector: every matrix U(-a, a) with
    a = sqrt(6 / (fan_in + fan_out)), every block whose name is in zero set to 0.
    shapes: list of (name, shape) in layout order."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in shapes:
        size = int(np.prod(shp))
        if name in zero:
            parts.append(np.zeros(size))
        else:
            fan_out, fan_in = shp[0], (shp[1] if len(shp) > 1 else 1)
            a = np.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-a, a, size))
    return np.concatenate(parts)
