"""Pins of the contact oracle (compliance matrix, projected Gauss-Seidel,
motion correction; paper Sec. 6.2) against facts that do not come from the
oracle itself: hand-computed iterates, an iterative solver in place of the
direct one, closed forms of special cases and the conditions that define the
answer."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import assembly, contact, solve, step

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pgs_small.json")


def _system(name, seed=0):
    w = synth.make(name)
    q, v = synth.random_state(w, 0.002, seed)
    ref = step.assemble(w, q, v)
    return w, ref


def test_pgs_hand_iterates():
    g = json.load(open(GOLDEN))
    for case in g["cases"]:
        W = np.array(case["W"], dtype=np.float64)
        c = np.array(case["c"], dtype=np.float64)
        for s, it in enumerate(case["iterates"]):
            lam = contact.pgs(W, c, s + 1)
            assert np.allclose(lam, it, rtol=0, atol=1e-15), (case["name"], s, lam)
        lam = contact.pgs(W, c, 60)
        assert np.allclose(lam, case["limit"], rtol=0, atol=1e-12), case["name"]
        assert contact.lcp_violation(W, c, lam) <= 1e-12


def test_compliance_of_all_dofs_is_the_inverse():
    # H = I (one constraint per DOF): W = A^{-1}, so W A = I
    w, ref = _system("tiny_hex")
    n = w.n_dofs
    H = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    W, Z = contact.compliance(n, ref.pat.row_ptr, ref.pat.col_idx, ref.vals, H)
    A = assembly.csr_to_dense(n, ref.pat.row_ptr, ref.pat.col_idx, ref.vals)
    assert np.abs(W @ A - np.eye(n)).max() <= 1e-9
    assert np.array_equal(W, Z)


def test_compliance_diagonal_closed_form():
    # A = diag(a): W_ab = sum_p h_ap h_bp / a_p
    w, _ = _system("tet_beam")
    n = w.n_dofs
    H, _ = synth.contact_constraints(w, 12, 3)
    a = np.random.default_rng(4).uniform(1.0, 3.0, n)
    rp, ci = np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)
    W, _ = contact.compliance(n, rp, ci, a, H)
    Hd = contact.h_dense(n, H)
    k = Hd.shape[0]
    Wc = np.zeros((k, k))
    for i in range(k):
        for j in range(k):
            Wc[i, j] = sum(Hd[i, p] * Hd[j, p] / a[p] for p in np.flatnonzero(Hd[i] * Hd[j]))
    assert np.abs(W - Wc).max() <= 1e-14 * np.abs(Wc).max()


@pytest.mark.parametrize("name,solver", [("tet_beam", "dense"), ("tet_beam", "banded")])
def test_compliance_against_iterative_solves(name, solver):
    # column b of W is the constraint response H x to the unit multiplier
    # force H^T e_b, with x from Jacobi-PCG instead of a Cholesky factor
    w, ref = _system(name)
    n = w.n_dofs
    p = ref.pat
    H, _ = synth.contact_constraints(w, 16, 5)
    W, Z = contact.compliance(n, p.row_ptr, p.col_idx, ref.vals, H, solver)
    Hd = contact.h_dense(n, H)
    for b in range(Hd.shape[0]):
        x, _, _ = solve.jacobi_pcg(p.row_ptr, p.col_idx, ref.vals, Hd[b].copy(), rel_tol=1e-11)
        col = contact.h_times(H, x)
        assert np.abs(col - W[:, b]).max() <= 1e-9 * np.abs(W).max()
        assert np.abs(x - Z[:, b]).max() <= 1e-9 * np.abs(Z).max()
    assert np.abs(W - W.T).max() <= 1e-12 * np.abs(W).max()
    assert np.linalg.eigvalsh(0.5 * (W + W.T)).min() > 0


def test_pgs_converges_to_the_lcp_solution():
    w, ref = _system("tet_beam")
    p = ref.pat
    H, _ = synth.contact_constraints(w, 20, 6)
    W, _ = contact.compliance(w.n_dofs, p.row_ptr, p.col_idx, ref.vals, H)
    rng = np.random.default_rng(7)
    # all constraints active: the answer solves W lambda = c
    lam_star = rng.uniform(0.5, 1.5, 20)
    c = W @ lam_star
    lam = contact.pgs(W, c, 20000)
    assert np.abs(lam - np.linalg.solve(W, c)).max() <= 1e-8 * np.abs(lam_star).max()
    # mixed signs: some constraints separate; the complementarity conditions hold
    c = rng.standard_normal(20) * np.abs(W).max()
    lam = contact.pgs(W, c, 20000)
    assert (lam == 0).any() and (lam > 0).any()
    assert contact.lcp_violation(W, c, lam) <= 1e-8


def test_contact_solve_kkt_and_constraints():
    # exact compliance: the corrected x satisfies A x + H^T lambda = b, active
    # constraints hold with equality and the others are not violated
    w, ref = _system("tet_beam")
    n = w.n_dofs
    p = ref.pat
    H, delta = synth.contact_constraints(w, 24, 8)
    W, _ = contact.compliance(n, p.row_ptr, p.col_idx, ref.vals, H)
    x_free = contact.solve_many(n, p.row_ptr, p.col_idx, ref.vals, ref.b)
    # put the obstacle where about half of the constraints are violated
    hx = contact.h_times(H, x_free)
    delta = hx - np.abs(hx).max() * 0.5 * delta
    x, xf, lam = contact.contact_solve(n, p.row_ptr, p.col_idx, ref.vals, ref.b, H, delta, W, 20000)
    assert np.abs(xf - x_free).max() == 0.0
    kkt = assembly.csr_matvec(p.row_ptr, p.col_idx, ref.vals, x) + contact.ht_times(n, H, lam) - ref.b
    assert np.abs(kkt).max() <= 1e-9 * np.abs(ref.b).max()
    g = contact.h_times(H, x) - delta
    scale = np.abs(delta).max()
    assert (lam > 0).sum() >= 3 and (lam == 0).sum() >= 3
    assert np.abs(g[lam > 0]).max() <= 1e-8 * scale
    assert g.max() <= 1e-8 * scale
