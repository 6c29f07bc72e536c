"""Direct and iterative reference solves of A x = b (oracle).

The paper solves the assembled system with a CG preconditioned by a stale
LDL^T factor (Sec. 3.3, Sec. 5).  The preconditioner changes only how fast CG
reaches the solution, so the oracle uses plain solves whose result is the
solution itself: dense Cholesky (small systems), banded Cholesky in the
natural node order (mid-size beams), LU for complex-step runs, and an FP64
Jacobi-PCG (any size, residual-certified).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .assembly import csr_matvec, csr_to_dense


def dense_cholesky_solve(n, row_ptr, col_idx, vals, b):
    """x = A^{-1} b through a dense Cholesky factor (A must be SPD)."""
    A = csr_to_dense(n, row_ptr, col_idx, vals)
    c = sla.cho_factor(A, lower=True)
    return sla.cho_solve(c, b)


def dense_lu_solve(n, row_ptr, col_idx, vals, b):
    """x = A^{-1} b through LU (works for complex-perturbed systems)."""
    A = csr_to_dense(n, row_ptr, col_idx, vals)
    return np.linalg.solve(A, b)


def bandwidth(row_ptr, col_idx):
    rows = np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))
    return int(np.max(np.abs(col_idx.astype(np.int64) - rows))) if rows.size else 0


def banded_cholesky_solve(n, row_ptr, col_idx, vals, b):
    """x = A^{-1} b through a banded Cholesky factor in the natural order."""
    u = bandwidth(row_ptr, col_idx)
    ab = np.zeros((u + 1, n))
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    up = col_idx >= rows
    # upper storage: ab[u + i - j, j] = A[i, j] for i <= j
    np.add.at(ab, (u + rows[up] - col_idx[up], col_idx[up]), vals[up])
    return sla.solveh_banded(ab, b, lower=False)


def jacobi_pcg(row_ptr, col_idx, vals, b, rel_tol=1e-12, max_it=100000, x0=None,
               time_limit=None):
    """Hestenes-Stiefel CG with a diagonal (Jacobi) preconditioner, FP64.

    Stops when ||b - A x|| / ||b|| <= rel_tol, with the residual recomputed
    from scratch when the recursive one says so.  Returns (x, iterations,
    relative residual).
    """
    import time
    t0 = time.perf_counter()
    n = b.size
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    diag = np.zeros(n)
    on = col_idx == rows
    np.add.at(diag, rows[on], vals[on])
    dinv = 1.0 / diag
    x = np.zeros(n) if x0 is None else x0.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros(n), 0, 0.0
    r = b - csr_matvec(row_ptr, col_idx, vals, x)
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < max_it:
        Ap = csr_matvec(row_ptr, col_idx, vals, p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        if np.linalg.norm(r) <= rel_tol * bn:
            r = b - csr_matvec(row_ptr, col_idx, vals, x)
            if np.linalg.norm(r) <= rel_tol * bn:
                break
        if time_limit is not None and time.perf_counter() - t0 > time_limit:
            break
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    res = np.linalg.norm(b - csr_matvec(row_ptr, col_idx, vals, x)) / bn
    return x, it, res
