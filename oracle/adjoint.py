"""Reverse-mode (adjoint) recursion of the implicit step (oracle).

Not in the paper: the gradient of a loss of the final state with respect to
per-element Young's moduli and the initial state.  Differentiating one step
(q+, v+) = (q + h v + h^2 a, v + h a) with A(q) a = b(q, v) gives, for the
incoming adjoints (lq+, lv+) = (dL/dq+, dL/dv+):

    abar = h lv+ + h^2 lq+            (fixed DOFs zeroed)
    A mu = abar                       (A is symmetric)
    lv   = lv+ + h lq+ - alpha M mu - (beta + h) K mu
    lq   = lq+ - K mu - (beta + h) T(q)[mu, v+]
    dL/dE_e += -(1/E_e) [mu_e . f_e + (beta + h) mu_e . K_e v+_e]

where T(q)[mu, w] = d/de K(q + e mu) w (third derivative of the stored energy)
and K, M here are the full (unconstrained) element sums; f and K are linear
in E at fixed nu, which gives the E term.  The oracle takes T by complex step
through its own element routines and checks the whole recursion against a
complex-step derivative of the complete rollout.
"""
from __future__ import annotations

import numpy as np

from . import assembly
from .step import assemble, element_data, pattern, rollout, solve_system

CS_EPS = 1e-30


def _elem_matvec(w, Ke, x):
    nen = w.conn.shape[1]
    xe = x.reshape(-1, 3)[w.conn].reshape(-1, 3 * nen)
    return np.einsum("eij,ej->ei", Ke, xe).reshape(-1, nen, 3)


def third_derivative(w, q, E, mu, wv):
    """T(q)[mu, w] = d/de (K(q + e mu) w) by complex step."""
    ed = element_data(w, q + 1j * CS_EPS * mu, E)
    Kw = assembly.assemble_vector(w.n_dofs, w.conn, _elem_matvec(w, ed.K, wv))
    return Kw.imag / CS_EPS


def adjoint_rollout(w, E, states, lam_qT, lam_vT, solver="dense"):
    """Run the recursion backwards over the stored states (q_n, v_n), n=0..N.

    Returns (dL/dE [E], dL/dq0 [n], dL/dv0 [n]).
    """
    if w.material not in (0, 1):
        raise ValueError("the adjoint recursion covers the neo-Hookean and St Venant-Kirchhoff "
                         "materials (f = dPsi/dq, K its Hessian)")
    pat = pattern(w)
    fixed = w.fixed.astype(bool)
    h, al, be = w.h, w.alpha, w.beta
    dE = np.zeros(w.n_elems)
    lq, lv = lam_qT.astype(np.float64).copy(), lam_vT.astype(np.float64).copy()
    nen = w.conn.shape[1]
    for n in reversed(range(len(states) - 1)):
        q, v = states[n]
        v1 = states[n + 1][1]
        sysm = assemble(w, q, v, E, pat)
        abar = h * lv + h * h * lq
        abar[fixed] = 0.0
        sysm.b = abar
        mu = solve_system(sysm, solver)
        ed = sysm.ed
        Kmu = assembly.assemble_vector(w.n_dofs, w.conn, _elem_matvec(w, ed.K, mu))
        Mmu = assembly.assemble_vector(w.n_dofs, w.conn, _elem_matvec(w, ed.M, mu))
        T = third_derivative(w, q, E, mu, v1)
        mu_e = mu.reshape(-1, 3)[w.conn].reshape(-1, 3 * nen)
        v1_e = v1.reshape(-1, 3)[w.conn].reshape(-1, 3 * nen)
        muf = np.sum(mu_e * ed.f.reshape(-1, 3 * nen), axis=1)
        muKv = np.einsum("ei,eij,ej->e", mu_e, ed.K, v1_e)
        dE += -(muf + (be + h) * muKv) / E
        lv, lq = lv + h * lq - al * Mmu - (be + h) * Kmu, lq - Kmu - (be + h) * T
    return dE, lq, lv


def loss_target(qT, q_target):
    d = qT - q_target
    return np.sum(d * d)


def rollout_loss_complex_step(w, E, q0, v0, q_target, nsteps, dE=None, dq0=None, dv0=None):
    """Directional derivative of L = ||q_T - q_target||^2 along (dE, dq0, dv0)
    by complex step through the complete rollout (LU solves)."""
    Ec = E + 1j * CS_EPS * (np.zeros_like(E) if dE is None else dE)
    qc = q0 + 1j * CS_EPS * (np.zeros_like(q0) if dq0 is None else dq0)
    vc = v0 + 1j * CS_EPS * (np.zeros_like(v0) if dv0 is None else dv0)
    states = rollout(w, qc, vc, nsteps, Ec, solver="lu")
    d = states[-1][0] - q_target
    return np.sum(d * d).imag / CS_EPS
