"""Contact through Lagrange multipliers (oracle): compliance matrix,
projected Gauss-Seidel and motion correction -- TEST INFRASTRUCTURE ONLY.

Sec. 6.2 solves contact in three stages around the same linear system as the
free step: a free motion A x_free = b; a constraint resolution on the
compliance matrix W = H A^{-1} H^T (Eq. "KKT", one deformable object), whose
complementarity problem is solved by projected Gauss-Seidel; and a motion
correction with one more solve of A.  Sec. 7.4 builds W with the stale
(asynchronous) preconditioner and a solver for many right-hand sides, so the
matrix inverted there is the factored snapshot A_t0; the oracle inverts the
snapshot it is given, directly.

Signs (reading R19): the KKT system and the printed correction disagree on
the sign of H for the first object.  Here the correction is taken as printed,
    x = x_free - A^{-1} H^T lambda,
so that H x = H x_free - W lambda.  With the constraint H x <= delta and
lambda >= 0, the complementarity problem is
    lambda >= 0,  W lambda - c >= 0,  lambda . (W lambda - c) = 0,
    c = H x_free - delta,
and active constraints (lambda_i > 0) end with (H x)_i = delta_i when W is
built with A itself.

H is a k x n CSR matrix given as (row_ptr, col, val).  Every function is
plain and unblocked.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import solve
from .assembly import csr_to_dense


def h_dense(n, H):
    """The k x n constraint matrix as a dense array (duplicates summed)."""
    row_ptr, col, val = H
    k = row_ptr.size - 1
    D = np.zeros((k, n))
    for a in range(k):
        for p in range(row_ptr[a], row_ptr[a + 1]):
            D[a, col[p]] += val[p]
    return D


def solve_many(n, row_ptr, col_idx, vals, B, solver="dense"):
    """X = A^{-1} B for the columns of B (one factorisation of A, dense or
    banded Cholesky in the natural order)."""
    if solver == "dense":
        A = csr_to_dense(n, row_ptr, col_idx, vals)
        return sla.cho_solve(sla.cho_factor(A, lower=True), B)
    return solve.banded_cholesky_solve(n, row_ptr, col_idx, vals, B)


def compliance(n, row_ptr, col_idx, vals, H, solver="dense"):
    """Sec. 6.2 constraint resolution: W = H A^{-1} H^T, with Z = A^{-1} H^T
    obtained as one solve with the k columns of H^T as right-hand sides.
    Returns (W, Z); Z is n x k."""
    Hd = h_dense(n, H)
    Z = solve_many(n, row_ptr, col_idx, vals, Hd.T.copy(), solver)
    return Hd @ Z, Z


def pgs(W, c, sweeps, lam0=None):
    """Projected Gauss-Seidel for lambda >= 0, W lambda - c >= 0,
    lambda . (W lambda - c) = 0 (Sec. 6.2 names the method; the update is the
    textbook one): each sweep visits the constraints in index order and sets
        lambda_i <- max(0, lambda_i - ((W lambda)_i - c_i) / W_ii)
    using the values already updated in this sweep."""
    k = c.size
    lam = np.zeros(k) if lam0 is None else np.array(lam0, dtype=np.float64)
    for _ in range(sweeps):
        for i in range(k):
            r = W[i] @ lam
            lam[i] = max(0.0, lam[i] - (r - c[i]) / W[i, i])
    return lam


def lcp_violation(W, c, lam):
    """Largest violation of the complementarity conditions: negative lambda,
    negative slack W lambda - c, and |lambda_i * slack_i|, each relative to
    the scale of c (0 for an exact solution)."""
    s = W @ lam - c
    scale = max(np.abs(c).max(), 1e-300)
    lam_scale = scale / max(np.abs(np.diag(W)).max(), 1e-300)
    return max(float(np.maximum(-lam, 0).max()) / lam_scale,
               float(np.maximum(-s, 0).max()) / scale,
               float(np.abs(lam * s).max()) / (scale * lam_scale))


def ht_times(n, H, lam):
    """H^T lambda (n-vector)."""
    row_ptr, col, val = H
    out = np.zeros(n)
    for a in range(row_ptr.size - 1):
        for p in range(row_ptr[a], row_ptr[a + 1]):
            out[col[p]] += val[p] * lam[a]
    return out


def h_times(H, x):
    """H x (k-vector)."""
    row_ptr, col, val = H
    k = row_ptr.size - 1
    out = np.zeros(k)
    for a in range(k):
        for p in range(row_ptr[a], row_ptr[a + 1]):
            out[a] += val[p] * x[col[p]]
    return out


def contact_solve(n, row_ptr, col_idx, vals, b, H, delta, W, sweeps, solver="dense"):
    """The three stages of Sec. 6.2 on one system A x = b with the constraint
    H x <= delta: free motion, projected Gauss-Seidel on the given compliance
    W (built from A or from a stale snapshot), motion correction with A.
    Returns (x, x_free, lambda)."""
    x_free = solve_many(n, row_ptr, col_idx, vals, b, solver)
    c = h_times(H, x_free) - delta
    lam = pgs(W, c, sweeps)
    dx = solve_many(n, row_ptr, col_idx, vals, ht_times(n, H, lam), solver)
    return x_free - dx, x_free, lam
