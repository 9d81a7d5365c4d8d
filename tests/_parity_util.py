"""Host-side measures of how far a GPU solution is from the oracle's, and the
bounds they must respect.  Test infrastructure: only the oracle and numpy are
used here.

Both solutions stop at ||r||/||b|| <= tol (Section 5), so they need not agree
to tol themselves; how far apart they may be is set by the conditioning:

* 2-norm.  x - x_o = A^{-1} (r_o - r) with r = b - A x, r_o = b - A x_o, so
  ||x - x_o|| <= (||r|| + ||r_o||) / lambda_min(A).  lambda_min(A) is bounded
  below by Gershgorin's min_i (a_ii - sum_{j != i} |a_ij|), which for the
  synthetic matrices (a weighted graph Laplacian plus a diagonal shift) is the
  shift itself; for the Dirichlet 5-point Laplacian on an m x m grid the
  closed form 8 sin^2(pi / (2 (m + 1))) is used.
* Energy norm.  With the preconditioner M = L L^T and the eigenvalues
  lambda_min, lambda_max of M^{-1} A, (1/lambda_max) M^{-1} <= A^{-1} <=
  (1/lambda_min) M^{-1}, hence
      ||x - x_o||_A / ||x_o||_A <= sqrt(kappa) ||r - r_o||_{M^-1} / ||b - r_o||_{M^-1},
  where kappa = lambda_max/lambda_min is estimated from the oracle's CG
  coefficients by the Lanczos tridiagonal matrix (Section 5, after Saad).
  Ritz values lie inside the spectrum, so that estimate can only be low; the
  tests allow a factor of 2 for it and for the rounding of the host
  residuals.
"""
from __future__ import annotations

import math

import numpy as np

import oracle


def gershgorin_lower(A) -> float:
    """min_i (a_ii - sum_{j != i} |a_ij|): a lower bound of lambda_min(A)."""
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    diag = np.zeros(A.n)
    off = np.zeros(A.n)
    on = rows == A.col
    np.add.at(diag, rows[on], A.val[on])
    np.add.at(off, rows[~on], np.abs(A.val[~on]))
    return float(np.min(diag - off))


def lambda_min_lower(A, name: str) -> float:
    """A rigorous lower bound of the smallest eigenvalue of the workload's matrix
    (invariant under the symmetric permutation)."""
    if name.startswith("laplace2d_"):
        m = int(name.split("_")[1])
        return 8.0 * math.sin(math.pi / (2 * (m + 1))) ** 2
    g = gershgorin_lower(A)
    assert g > 0.0, f"no Gershgorin bound for {name}"
    return g * (1.0 - 1e-9)


def solution_report(Ap, lval, bp, x, ref, lam_min: float, tol: float) -> dict:
    """Distance of x from the oracle solution ref.x and its two bounds."""
    xo = ref.x
    r = bp - oracle.spmv(Ap, x)
    ro = bp - oracle.spmv(Ap, xo)
    e = x - xo
    nxo = float(np.linalg.norm(xo))
    err2 = float(np.linalg.norm(e)) / nxo
    bound2 = (float(np.linalg.norm(r)) + float(np.linalg.norm(ro))) / (lam_min * nxo)
    dr = r - ro
    bo = bp - ro
    lo, hi, kappa = oracle.lanczos_kappa(ref.alphas, ref.betas)
    errA = math.sqrt(max(oracle.dot(e, oracle.spmv(Ap, e)), 0.0) /
                     oracle.dot(xo, oracle.spmv(Ap, xo)))
    boundA = math.sqrt(kappa) * math.sqrt(max(oracle.dot(dr, oracle.ic_apply(Ap, lval, dr)), 0.0) /
                                          oracle.dot(bo, oracle.ic_apply(Ap, lval, bo)))
    return {"err2": err2, "bound2": bound2, "errA": errA, "boundA": boundA,
            "kappa_lanczos": kappa, "two_kappa_tol": 2.0 * kappa * tol,
            "relres_true": float(np.linalg.norm(r) / np.linalg.norm(bp)),
            "relres_true_oracle": float(np.linalg.norm(ro) / np.linalg.norm(bp))}


def history_sensitivity(Ap, lval, bp, tol: float, m: int, seeds=(0, 1, 2)) -> float:
    """How far the oracle's own residual history moves when b is perturbed by
    one ulp in about two thirds of its entries (random signs): the largest
    history_deviation over the first m entries across a few perturbations.
    The CG recurrence amplifies any rounding difference at the rate set by
    the conditioning (and by transient growth of ||r||), so no two
    implementations that round differently can agree more closely than
    this."""
    ref = oracle.pcg(Ap, lval, bp, tol=tol, maxit=max(m, 1) + 5000)
    worst = 0.0
    for sd in seeds:
        rng = np.random.default_rng(sd)
        bq = bp * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 0.0, 1.0], size=bp.size))
        other = oracle.pcg(Ap, lval, bq, tol=tol, maxit=max(m, 1) + 5000)
        k = min(m, ref.iters + 1, other.iters + 1)
        worst = max(worst, history_deviation(other.history, ref.history, k))
    return worst


def history_deviation(hist, ref_hist, m: int) -> float:
    """max_k |h_k - h^o_k| / h^o_k over the first m entries."""
    h = np.asarray(hist[:m], dtype=np.float64)
    o = np.asarray(ref_hist[:m], dtype=np.float64)
    return float(np.max(np.abs(h - o) / o))
