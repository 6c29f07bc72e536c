"""One implicit step of the paper's method, FP64 (oracle).

Sec. 3.2: Newton's law M a = p - F(q, v) (Eq. "newton's law"), backward Euler
v+ = v + h a, q+ = q + h v+ (Eq. "implicit integration"), one first-order
Taylor expansion of F (Eq. "taylor expansion") with Rayleigh damping
B = alpha M + beta K, giving A a = b with
    A = (1 + h alpha) M + h (beta + h) K            (Eq. "dynamic equation2").
The right-hand side is printed three different ways in the paper; the reading
used here (R1) follows from the Taylor expansion with F = f(q) + B v:
    b = p - f(q) - alpha M v - (beta + h) K(q) v,
which reduces to the Sec. 4.2 form when alpha = beta = 0.  Fixed DOFs follow
Sec. 6.1: rows/cols removed, 1 on the diagonal, and b_d = 0 (reading R6), so
a_d = 0 and fixed nodes keep their initial position and velocity.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import assembly, elements, solve


@dataclass
class Pattern:
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    tmap: np.ndarray
    fixed_dofs: np.ndarray
    diag_slots: np.ndarray

    @property
    def nnz(self):
        return self.col_idx.size


def pattern(w) -> Pattern:
    rp, ci, tm, fd, ds = assembly.build_pattern(w.n_dofs, w.conn, w.fixed)
    return Pattern(w.n_dofs, rp, ci, tm, fd, ds)


@dataclass
class ElementData:
    f: np.ndarray        # [E, nen, 3] internal force
    K: np.ndarray        # [E, 3nen, 3nen] tangent stiffness
    M: np.ndarray        # [E, 3nen, 3nen] consistent mass (blocks M_ab I)
    p_grav: np.ndarray   # [E, nen, 3] gravity load M (1 (x) g)


def element_data(w, q, E=None) -> ElementData:
    E = w.E if E is None else E
    nen = w.conn.shape[1]
    Xe = w.X[w.conn]
    xe = q.reshape(-1, 3)[w.conn]
    f, K = elements.element_force_stiffness(w.elem_type, Xe, xe, E, w.nu, w.material,
                                            w.mr_c01_share)
    K = K.reshape(-1, 3 * nen, 3 * nen)
    m = elements.element_mass(w.elem_type, Xe, w.rho)
    M = np.einsum("eab,ij->eaibj", m, np.eye(3)).reshape(-1, 3 * nen, 3 * nen)
    p_grav = np.einsum("eab,j->eaj", m, w.gravity)
    return ElementData(f, K, M, p_grav)


@dataclass
class System:
    pat: Pattern
    vals: np.ndarray     # A in CSR order
    b: np.ndarray
    ed: ElementData


def element_lhs(w, ed):
    return (1.0 + w.h * w.alpha) * ed.M + w.h * (w.beta + w.h) * ed.K


def element_rhs(w, ed, v):
    """b_e = p_grav - f - alpha M v - (beta + h) K v (element vectors)."""
    nen = w.conn.shape[1]
    ve = v.reshape(-1, 3)[w.conn].reshape(-1, 3 * nen)
    Mv = np.einsum("eij,ej->ei", ed.M, ve)
    Kv = np.einsum("eij,ej->ei", ed.K, ve)
    be = ed.p_grav.reshape(-1, 3 * nen) - ed.f.reshape(-1, 3 * nen) - w.alpha * Mv - (w.beta + w.h) * Kv
    return be.reshape(-1, nen, 3)


def assemble(w, q, v, E=None, pat: Pattern | None = None) -> System:
    pat = pattern(w) if pat is None else pat
    ed = element_data(w, q, E)
    Ae = element_lhs(w, ed)
    vals = assembly.assemble_values(pat.nnz, pat.tmap, Ae, pat.diag_slots)
    b = assembly.assemble_vector(w.n_dofs, w.conn, element_rhs(w, ed, v))
    b = b + w.f_nodal.reshape(-1)
    b[w.fixed.astype(bool)] = 0.0
    return System(pat, vals, b, ed)


def solve_system(sysm: System, solver="dense", rel_tol=1e-12):
    p = sysm.pat
    if solver == "dense":
        return solve.dense_cholesky_solve(p.n, p.row_ptr, p.col_idx, sysm.vals, sysm.b)
    if solver == "lu":
        return solve.dense_lu_solve(p.n, p.row_ptr, p.col_idx, sysm.vals, sysm.b)
    if solver == "banded":
        return solve.banded_cholesky_solve(p.n, p.row_ptr, p.col_idx, sysm.vals, sysm.b)
    if solver == "pcg":
        x, _, _ = solve.jacobi_pcg(p.row_ptr, p.col_idx, sysm.vals, sysm.b, rel_tol)
        return x
    raise ValueError(solver)


def step(w, q, v, E=None, solver="dense", pat=None):
    """One step: returns (q+, v+, a)."""
    sysm = assemble(w, q, v, E, pat)
    a = solve_system(sysm, solver)
    v1 = v + w.h * a
    q1 = q + w.h * v1
    return q1, v1, a


def rollout(w, q0, v0, nsteps, E=None, solver="dense"):
    """States [(q_0, v_0), ..., (q_N, v_N)] of nsteps steps."""
    pat = pattern(w)
    states = [(q0, v0)]
    q, v = q0, v0
    for _ in range(nsteps):
        q, v, _ = step(w, q, v, E, solver, pat)
        states.append((q, v))
    return states


def default_solver(n):
    return "dense" if n <= 4000 else "banded"
