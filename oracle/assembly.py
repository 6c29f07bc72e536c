"""Triplet collection, pattern + map by comparison sort, and assembly (oracle).

Paper Sec. 4.1 collects element contributions as (row, col, value) triplets
in a fill order that depends only on the topology; Sec. 4.2 turns them into a
CSR matrix and a map C from each triplet to its CSR slot, so that later steps
only sum values through C.  Sec. 6.1 (projective constraints) drops the rows
and columns of fixed DOFs while C is built and puts 1 on their diagonal.

The oracle reaches the same pattern and map with a plain comparison sort
(``numpy.lexsort``) of the triplet keys, deliberately unlike a counting-sort
transpose, so the two constructions pin each other.

Canonical fill order (element-major): element e, then local row i = 3a + r,
then local column j = 3b + c, row-major over (i, j); global row
3 conn[e, a] + r, global column 3 conn[e, b] + c.
"""
from __future__ import annotations

import numpy as np


def triplet_keys(conn):
    """Global (row, col) of every element triplet in canonical order, flat."""
    nen = conn.shape[1]
    dof = (3 * conn[:, :, None].astype(np.int64) + np.arange(3)).reshape(-1, 3 * nen)
    rows = np.broadcast_to(dof[:, :, None], (conn.shape[0], 3 * nen, 3 * nen))
    cols = np.broadcast_to(dof[:, None, :], (conn.shape[0], 3 * nen, 3 * nen))
    return rows.reshape(-1), cols.reshape(-1)


def build_pattern(n_dofs, conn, fixed):
    """CSR pattern (row_ptr, col_idx) and the triplet -> CSR map.

    Triplets touching a fixed row or column are dropped (map = -1); each fixed
    DOF d contributes one structural entry (d, d).  Structural pattern: entries
    are kept whatever their numerical value.
    """
    fixed = np.asarray(fixed).astype(bool)
    rows, cols = triplet_keys(conn)
    keep = ~fixed[rows] & ~fixed[cols]
    fd = np.flatnonzero(fixed)
    all_r = np.concatenate([rows[keep], fd])
    all_c = np.concatenate([cols[keep], fd])
    order = np.lexsort((all_c, all_r))           # sort by row, then column
    sr, sc = all_r[order], all_c[order]
    new = np.ones(sr.size, dtype=bool)
    new[1:] = (sr[1:] != sr[:-1]) | (sc[1:] != sc[:-1])
    slot_sorted = np.cumsum(new) - 1               # CSR slot of each sorted key
    col_idx = sc[new].astype(np.int32)
    row_of_slot = sr[new]
    row_ptr = np.zeros(n_dofs + 1, dtype=np.int64)
    np.add.at(row_ptr, row_of_slot + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    slot = np.empty(sr.size, dtype=np.int64)
    slot[order] = slot_sorted
    tmap = np.full(rows.size, -1, dtype=np.int64)
    tmap[np.flatnonzero(keep)] = slot[: int(keep.sum())]
    diag_slots = slot[int(keep.sum()):]
    return row_ptr, col_idx, tmap.astype(np.int32), fd, diag_slots


def assemble_values(nnz, tmap, values, fixed_diag_slots):
    """Sum element triplet values into CSR slots through the map (FP64)."""
    keep = tmap >= 0
    vals = _segment_add(tmap[keep], values.reshape(-1)[keep], nnz)
    vals[fixed_diag_slots] += 1.0
    return vals


def _segment_add(index, values, size):
    """out[k] = sum of values[t] over t with index[t] == k (FP64 or complex)."""
    if np.iscomplexobj(values):
        return (np.bincount(index, weights=values.real, minlength=size)
                + 1j * np.bincount(index, weights=values.imag, minlength=size))
    return np.bincount(index, weights=values, minlength=size).astype(np.float64)


def assemble_vector(n_dofs, conn, ve):
    """Scatter-add element vectors ve [E, nen, 3] into a global vector."""
    dof = (3 * conn[:, :, None].astype(np.int64) + np.arange(3)).reshape(-1)
    return _segment_add(dof, ve.reshape(-1), n_dofs)


def csr_to_dense(n, row_ptr, col_idx, vals):
    A = np.zeros((n, n), dtype=vals.dtype)
    for i in range(n):
        A[i, col_idx[row_ptr[i]:row_ptr[i + 1]]] += vals[row_ptr[i]:row_ptr[i + 1]]
    return A


def csr_matvec(row_ptr, col_idx, vals, x):
    """y = A x row by row (plain CSR definition), vectorised with a segment sum."""
    prod = vals * x[col_idx]
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    return _segment_add(rows, prod, n)
