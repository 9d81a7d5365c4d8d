"""Serial FP64 CPU oracle for block-multicolored ICCG — TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never imports, links or calls
it, and this package imports nothing from the product library: the two share
only the seeded input generators in ``synth``.

The arithmetic lives in ``oracle.c`` (plain serial C, FP64, built with
``-ffp-contract=off``); this module marshals numpy arrays into it and adds a
few closed-form statistics written directly from their definitions in the
paper:

* Gini coefficient of block sizes (Section 7.3),
* B_max, B_max/B_avg, C_max/C_avg (Section 7.3, Table 6),
* modularity, Eq. (1), and CPM quality, Eq. (2) (Section 4),
* Lanczos condition-number estimate from the CG coefficients (Section 5,
  after Saad's Iterative Methods, Section 6.7.3).

Parity status of each function is recorded in the module docstrings below and
in the design notes; every function here is pinned by a ``-m "not gpu"`` test
except where marked "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile liboracle.so with gcc (serial, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
           "-D_POSIX_C_SOURCE=199309L", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    c_int, c_dbl, c_u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    ip = ctypes.POINTER(c_int)
    dp = ctypes.POINTER(c_dbl)
    lib.or_abmc.argtypes = [c_int, _i32p, _i32p, c_int, _i32p]
    lib.or_abmc.restype = c_int
    lib.or_color_blocks.argtypes = [c_int, _i32p, _i32p, c_int, _i32p, _i32p]
    lib.or_color_blocks.restype = c_int
    lib.or_order.argtypes = [c_int, c_int, _i32p, _i32p, c_int, _i32p, _i32p, _i32p]
    lib.or_order.restype = None
    lib.or_permute.argtypes = [c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _i32p, _f64p]
    lib.or_permute.restype = None
    lib.or_ic0.argtypes = [c_int, _i32p, _i32p, _f64p, _f64p]
    lib.or_ic0.restype = c_int
    for fn in (lib.or_forward, lib.or_backward, lib.or_ic_apply):
        fn.argtypes = [c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        fn.restype = None
    lib.or_spmv.argtypes = [c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
    lib.or_spmv.restype = None
    lib.or_dot.argtypes = [c_int, _f64p, _f64p]
    lib.or_dot.restype = c_dbl
    lib.or_pcg.argtypes = [c_int, _i32p, _i32p, _f64p, ctypes.c_void_p, _f64p, _f64p,
                           c_dbl, c_int, ip, dp, dp, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.c_void_p]
    lib.or_pcg.restype = c_int
    lib.or_leiden.argtypes = [c_int, _i32p, _i32p, c_int, c_dbl, c_dbl, c_int, c_u64, _i32p]
    lib.or_leiden.restype = c_int
    lib.or_sort_blocks.argtypes = [c_int, c_int, _i32p]
    lib.or_sort_blocks.restype = None
    lib.or_splitmix64_draws.argtypes = [c_u64, c_int, _u64p]
    lib.or_splitmix64_draws.restype = c_u64
    _lib = lib
    return lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# RNG (SplitMix64) -- exposed so that its published test vector can pin it
# --------------------------------------------------------------------------
def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().or_splitmix64_draws(seed, count, out)
    return out


# --------------------------------------------------------------------------
# ordering (Section 3, Section 6.1, Section 7.1)
# --------------------------------------------------------------------------
def abmc_blocks(A, s: int) -> np.ndarray:
    """ABMC block id of every node for block size s (Section 3)."""
    block_of = np.zeros(A.n, dtype=np.int32)
    _load().or_abmc(A.n, _i32(A.rowptr), _i32(A.col), int(s), block_of)
    return block_of


def leiden_blocks(A, quality: str, gamma: float, beta: float = 0.01, n_iter: int = 2,
                  seed: int = 42) -> np.ndarray:
    """Leiden communities of the pattern graph (Section 4, Section 7.1).

    quality is "modularity" (Eq. 1) or "cpm" (Eq. 2).  Communities are numbered
    in ascending order of their smallest node (not yet size-sorted).
    """
    q = {"modularity": 0, "cpm": 1}[quality]
    memb = np.zeros(A.n, dtype=np.int32)
    _load().or_leiden(A.n, _i32(A.rowptr), _i32(A.col), q, float(gamma), float(beta),
                      int(n_iter), int(seed), memb)
    return memb


def sort_blocks_by_size(block_of: np.ndarray) -> np.ndarray:
    """Renumber blocks by descending size, ties by smaller minimum node (Section 7.1)."""
    out = _i32(block_of).copy()
    nb = int(out.max()) + 1 if out.size else 0
    _load().or_sort_blocks(out.size, nb, out)
    return out


def color_blocks(A, block_of: np.ndarray) -> np.ndarray:
    """Greedy block coloring in ascending block id (Section 6.1)."""
    nb = int(block_of.max()) + 1 if block_of.size else 0
    color = np.zeros(nb, dtype=np.int32)
    _load().or_color_blocks(A.n, _i32(A.rowptr), _i32(A.col), nb, _i32(block_of), color)
    return color


@dataclass
class Ordering:
    perm: np.ndarray        # perm[new] = old
    block_ptr: np.ndarray   # n_b + 1
    color_ptr: np.ndarray   # n_c + 1

    @property
    def nblocks(self) -> int:
        return self.block_ptr.size - 1

    @property
    def ncolors(self) -> int:
        return self.color_ptr.size - 1


def color_major_order(A, block_of: np.ndarray, color_of_block: np.ndarray) -> Ordering:
    nb = color_of_block.size
    nc = int(color_of_block.max()) + 1 if nb else 0
    perm = np.zeros(A.n, dtype=np.int32)
    bp = np.zeros(nb + 1, dtype=np.int32)
    cp = np.zeros(nc + 1, dtype=np.int32)
    _load().or_order(A.n, nb, _i32(block_of), _i32(color_of_block), nc, perm, bp, cp)
    return Ordering(perm, bp, cp)


def order_abmc(A, s: int) -> Ordering:
    blocks = abmc_blocks(A, s)
    return color_major_order(A, blocks, color_blocks(A, blocks))


def order_leiden(A, quality: str, gamma: float, beta: float = 0.01, n_iter: int = 2,
                 seed: int = 42) -> Ordering:
    blocks = sort_blocks_by_size(leiden_blocks(A, quality, gamma, beta, n_iter, seed))
    return color_major_order(A, blocks, color_blocks(A, blocks))


def permute(A, perm: np.ndarray):
    """A' = P A P^T with sorted columns (perm[new] = old)."""
    from synth import CSR  # container type only
    prow = np.zeros(A.n + 1, dtype=np.int32)
    pcol = np.zeros(A.nnz, dtype=np.int32)
    pval = np.zeros(A.nnz, dtype=np.float64)
    _load().or_permute(A.n, _i32(A.rowptr), _i32(A.col), _f64(A.val), _i32(perm),
                       prow, pcol, pval)
    return CSR(A.n, prow, pcol, pval)


# --------------------------------------------------------------------------
# IC(0), substitutions, SpMV, PCG
# --------------------------------------------------------------------------
def ic0(A):
    """IC(0): returns (lval, breakdown_row).  lval has A's positions, lower part
    (diagonal included) filled, upper part zero; breakdown_row is -1 on success."""
    lval = np.zeros(A.nnz, dtype=np.float64)
    row = _load().or_ic0(A.n, _i32(A.rowptr), _i32(A.col), _f64(A.val), lval)
    return lval, int(row)


def forward(A, lval, r):
    y = np.zeros(A.n)
    _load().or_forward(A.n, _i32(A.rowptr), _i32(A.col), _f64(lval), _f64(r), y)
    return y


def backward(A, lval, y):
    z = np.zeros(A.n)
    _load().or_backward(A.n, _i32(A.rowptr), _i32(A.col), _f64(lval), _f64(y), z)
    return z


def ic_apply(A, lval, r):
    z = np.zeros(A.n)
    _load().or_ic_apply(A.n, _i32(A.rowptr), _i32(A.col), _f64(lval), _f64(r), z)
    return z


def spmv(A, x):
    y = np.zeros(A.n)
    _load().or_spmv(A.n, _i32(A.rowptr), _i32(A.col), _f64(A.val), _f64(x), y)
    return y


def dot(a, b) -> float:
    a, b = _f64(a), _f64(b)
    return float(_load().or_dot(a.size, a, b))


@dataclass
class PCGResult:
    status: int            # 0 converged, 1 maxit, 2 breakdown of (p, q)
    iters: int
    relres: float          # recursive ||r||/||b||
    relres_true: float     # ||b - A x|| / ||b||
    x: np.ndarray
    history: np.ndarray    # relres after each iteration, [0] = initial
    alphas: np.ndarray
    betas: np.ndarray
    phase_s: np.ndarray    # seconds: forward, backward, SpMV, other


def pcg(A, lval, b, tol: float = 1e-8, maxit: int = 10000, x0=None) -> PCGResult:
    """PCG with M = L L^T (lval from ic0) or M = I (lval=None), Section 5."""
    n = A.n
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit + 1)
    al = np.zeros(max(maxit, 1))
    be = np.zeros(max(maxit, 1))
    ph = np.zeros(4)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    rt = ctypes.c_double(0.0)
    lv = None if lval is None else _f64(lval)
    st = _load().or_pcg(n, _i32(A.rowptr), _i32(A.col), _f64(A.val),
                        None if lv is None else lv.ctypes.data, _f64(b), x, float(tol),
                        int(maxit), ctypes.byref(it), ctypes.byref(rr), ctypes.byref(rt),
                        hist.ctypes.data, al.ctypes.data, be.ctypes.data, ph.ctypes.data)
    k = it.value
    return PCGResult(int(st), k, rr.value, rt.value, x, hist[:k + 1].copy(), al[:k].copy(),
                     be[:max(k - 1, 0)].copy(), ph)


def lanczos_kappa(alphas: np.ndarray, betas: np.ndarray):
    """Condition-number estimate from CG coefficients (Section 5, after Saad).

    T is the Lanczos tridiagonal matrix implied by CG:
      T_00 = 1/alpha_0,  T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
      T_{j-1,j} = T_{j,j-1} = sqrt(beta_{j-1}) / alpha_{j-1}.
    Returns (lambda_min, lambda_max, kappa) of T.
    """
    k = len(alphas)
    if k == 0:
        return float("nan"), float("nan"), float("nan")
    m = min(k, len(betas) + 1)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j]
        if j > 0:
            T[j, j] += betas[j - 1] / alphas[j - 1]
            T[j, j - 1] = T[j - 1, j] = np.sqrt(betas[j - 1]) / alphas[j - 1]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1]), float(ev[-1] / ev[0])


# --------------------------------------------------------------------------
# statistics (Section 7.3) and quality functions (Section 4)
# --------------------------------------------------------------------------
def gini(sizes) -> float:
    """G = sum_i sum_j |s_i - s_j| / (2 n_b^2 mean(s)) -- Section 7.3."""
    s = np.asarray(sizes, dtype=np.float64)
    nb = s.size
    if nb == 0:
        return 0.0
    total = 0.0
    for i in range(nb):
        total += np.abs(s[i] - s).sum()
    return float(total / (2.0 * nb * nb * s.mean()))


def block_stats(order: Ordering) -> dict:
    """n_b, n_c, G, B_max, B_max/B_avg, C_max/C_avg (Section 7.3, Table 6)."""
    bs = np.diff(order.block_ptr)
    rows_per_color = np.array([order.block_ptr[order.color_ptr[c + 1]] -
                               order.block_ptr[order.color_ptr[c]]
                               for c in range(order.ncolors)], dtype=np.float64)
    return {
        "n_b": int(bs.size),
        "n_c": int(order.ncolors),
        "gini": gini(bs),
        "B_max": int(bs.max()),
        "B_max_over_avg": float(bs.max() / bs.mean()),
        "C_max_over_avg": float(rows_per_color.max() / rows_per_color.mean()),
    }


def quality(A, membership, kind: str, gamma: float) -> float:
    """Eq. (1) (kind="modularity") or Eq. (2) (kind="cpm") of a partition of the
    unweighted pattern graph of A, summed over ordered pairs (i, j) including
    i = j, with m the number of undirected edges and k_i the degree."""
    memb = np.asarray(membership)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    off = rows != A.col
    ri, cj = rows[off], A.col[off]
    m2 = float(ri.size)                      # 2m
    k = np.bincount(ri, minlength=A.n).astype(np.float64)
    q = 0.0
    # sum over same-community ordered pairs of A_ij
    q += float(np.sum(memb[ri] == memb[cj]))
    # minus the null-model / constant term over same-community ordered pairs
    for c in np.unique(memb):
        sel = memb == c
        if kind == "modularity":
            K = k[sel].sum()
            q -= gamma * K * K / m2
        else:
            N = float(sel.sum())
            q -= gamma * N * N
    return q / m2


def community_connected(A, membership) -> bool:
    """True iff every community induces a connected subgraph of the pattern graph."""
    memb = np.asarray(membership)
    n = A.n
    comp = np.full(n, -1, dtype=np.int64)
    ncomp = 0
    for start in range(n):
        if comp[start] >= 0:
            continue
        c = memb[start]
        stack = [start]
        comp[start] = ncomp
        while stack:
            v = stack.pop()
            for k in range(A.rowptr[v], A.rowptr[v + 1]):
                u = A.col[k]
                if comp[u] < 0 and memb[u] == c:
                    comp[u] = ncomp
                    stack.append(u)
        ncomp += 1
    # connected iff each community is exactly one component
    return ncomp == np.unique(memb).size
