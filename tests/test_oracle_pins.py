"""Pins of the FP64 oracle against facts outside itself.

Each test checks the oracle against a closed form, an invariant of continuum
mechanics, a textbook formula written independently, brute force, or a
complex-step derivative of the oracle's own forward rollout.  A dropped term,
a wrong sign or a transposed operand in the oracle fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import adjoint, assembly, elements, solve, step

MATS = [elements.NEO_HOOKEAN, elements.ST_VENANT_KIRCHHOFF]
MESHES = ["tiny_tet", "tiny_hex"]


def _elem(w, q):
    Xe = w.X[w.conn]
    xe = q.reshape(-1, 3)[w.conn]
    G, dV = elements.quadrature(w.elem_type, Xe)
    mu, lam = elements.lame(w.E, w.nu)
    return xe, G, dV, mu, lam


def _deformed(w, seed=5, scale=0.15):
    q, _ = synth.random_state(w, scale, seed)
    return q


# ---------------------------------------------------------------- elements

@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_stiffness_symmetric(mesh, mat):
    w = synth.make(mesh, material=mat)
    xe, G, dV, mu, lam = _elem(w, _deformed(w))
    K = elements.element_stiffness(xe, G, dV, mu, lam, mat)
    n = 3 * w.conn.shape[1]
    K = K.reshape(-1, n, n)
    assert np.abs(K - K.transpose(0, 2, 1)).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_translation_invariance(mesh, mat):
    """f(x + 1 t) = f(x) and K (1 (x) t) = 0 at any state."""
    w = synth.make(mesh, material=mat)
    xe, G, dV, mu, lam = _elem(w, _deformed(w))
    t = np.array([0.3, -0.7, 0.2])
    f0 = elements.element_force(xe, G, dV, mu, lam, mat)
    f1 = elements.element_force(xe + t, G, dV, mu, lam, mat)
    assert np.abs(f1 - f0).max() <= 1e-12 * np.abs(f0).max()
    K = elements.element_stiffness(xe, G, dV, mu, lam, mat)
    Kt = np.einsum("eaibj,j->eai", K, t)
    assert np.abs(Kt).max() <= 1e-11 * np.abs(K).max()
    # internal forces of an element sum to zero (no net force)
    assert np.abs(f0.sum(axis=1)).max() <= 1e-12 * np.abs(f0).max()


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_rotation_identity(mesh, mat):
    """Objectivity: f(R x) = R f(x); differentiated at R = I: K (W x) = W f."""
    w = synth.make(mesh, material=mat)
    xe, G, dV, mu, lam = _elem(w, _deformed(w))
    f = elements.element_force(xe, G, dV, mu, lam, mat)
    ang = 0.7
    R = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1.0]])
    R = R @ np.array([[1, 0, 0], [0, np.cos(0.4), -np.sin(0.4)], [0, np.sin(0.4), np.cos(0.4)]])
    fR = elements.element_force(xe @ R.T, G, dV, mu, lam, mat)
    assert np.abs(fR - f @ R.T).max() <= 1e-11 * np.abs(f).max()
    W = np.array([[0, -0.3, 0.5], [0.3, 0, -0.2], [-0.5, 0.2, 0]])
    K = elements.element_stiffness(xe, G, dV, mu, lam, mat)
    lhs = np.einsum("eaibj,ebj->eai", K, xe @ W.T)
    assert np.abs(lhs - f @ W.T).max() <= 1e-10 * np.abs(f).max()


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_force_is_energy_gradient_and_stiffness_is_force_jacobian(mesh, mat):
    """Central differences with O(eps^2) error: halving eps quarters the error."""
    w = synth.make(mesh, material=mat)
    xe, G, dV, mu, lam = _elem(w, _deformed(w))
    d = np.random.default_rng(0).standard_normal(xe.shape) * 1e-4
    f = elements.element_force(xe, G, dV, mu, lam, mat)
    K = elements.element_stiffness(xe, G, dV, mu, lam, mat)
    Kd = np.einsum("eaibj,ebj->eai", K, d)
    errs_K, errs_f = [], []
    for eps in (1e-1, 5e-2):
        fp = elements.element_force(xe + eps * d, G, dV, mu, lam, mat)
        fm = elements.element_force(xe - eps * d, G, dV, mu, lam, mat)
        errs_K.append(np.abs((fp - fm) / (2 * eps) - Kd).max())
        Ep = elements.element_energy(xe + eps * d, G, dV, mu, lam, mat)
        Em = elements.element_energy(xe - eps * d, G, dV, mu, lam, mat)
        errs_f.append(np.abs((Ep - Em) / (2 * eps) - np.einsum("eai,eai->e", f, d)).max())
    assert errs_K[1] <= 1e-3 * np.abs(Kd).max()
    assert 3.0 < errs_K[0] / errs_K[1] < 5.0
    assert 3.0 < errs_f[0] / errs_f[1] < 5.0


def _voigt_B(g):
    """Strain-displacement matrix (engineering shear) for gradients g [nen, 3]."""
    nen = g.shape[0]
    B = np.zeros((6, 3 * nen))
    for a in range(nen):
        gx, gy, gz = g[a]
        c = 3 * a
        B[0, c] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c] = gy; B[3, c + 1] = gx
        B[4, c + 1] = gz; B[4, c + 2] = gy
        B[5, c] = gz; B[5, c + 2] = gx
    return B


def _voigt_C(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2 * mu
    C[3:, 3:] = mu * np.eye(3)
    return C


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_rest_state_is_linear_elasticity(mesh, mat):
    """At F = I: f = 0 and K_e = sum_q dV B^T C B (textbook Voigt form)."""
    w = synth.make(mesh, material=mat)
    xe, G, dV, mu, lam = _elem(w, w.q0())
    f = elements.element_force(xe, G, dV, mu, lam, mat)
    K = elements.element_stiffness(xe, G, dV, mu, lam, mat)
    n = 3 * w.conn.shape[1]
    K = K.reshape(-1, n, n)
    assert np.abs(f).max() <= 1e-12 * np.abs(K).max() * 0.01
    C = _voigt_C(w.E[0], w.nu)
    for e in range(w.n_elems):
        Kref = sum(dV[e, q] * _voigt_B(G[e, q]).T @ C @ _voigt_B(G[e, q]) for q in range(G.shape[1]))
        assert np.abs(K[e] - Kref).max() <= 1e-12 * np.abs(Kref).max()


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_linear_in_young_modulus(mesh, mat):
    w = synth.make(mesh, material=mat)
    q = _deformed(w)
    f1, K1 = elements.element_matrices(w.elem_type, w.X, w.conn, q, w.E, w.nu, mat)
    f2, K2 = elements.element_matrices(w.elem_type, w.X, w.conn, q, 2.5 * w.E, w.nu, mat)
    assert np.allclose(f2, 2.5 * f1, rtol=1e-13, atol=1e-13 * np.abs(f1).max())
    assert np.allclose(K2, 2.5 * K1, rtol=1e-13, atol=1e-13 * np.abs(K1).max())


# ------------------------------------------------------------- geometry, mass

@pytest.mark.parametrize("mesh", ["tiny_tet", "tiny_hex", "hex_diff"])
def test_volume_and_mass_sums(mesh):
    w = synth.make(mesh)
    G, dV = elements.quadrature(w.elem_type, w.X[w.conn])
    box = np.prod(np.asarray(w.dims) * w.spacing)
    assert abs(dV.sum() - box) <= 1e-12 * box
    m = elements.element_mass(w.elem_type, w.X[w.conn], w.rho)
    assert abs(m.sum() - w.rho * box) <= 1e-12 * w.rho * box


def test_tet_mass_against_degree2_quadrature():
    """Consistent tet mass vs the 4-point (degree-2 exact) rule: independent."""
    w = synth.make("tiny_tet")
    Xe = w.X[w.conn]
    m = elements.element_mass(4, Xe, w.rho)
    a, b = 0.5854101966249685, 0.1381966011250105
    bary = np.array([[a, b, b, b], [b, a, b, b], [b, b, a, b], [b, b, b, a]])
    _, V = elements.tet_gradients(Xe)
    ref = w.rho * V[:, None, None] * np.einsum("qa,qb->ab", bary, bary)[None] / 4.0
    assert np.abs(m - ref).max() <= 1e-13 * np.abs(ref).max()


def test_hex_cube_mass_closed_form():
    """Cube: M = rho V / 216 x {8, 4, 2, 1} (tensor product of [2 1; 1 2]/6)."""
    Xe = synth.HEX_CORNERS[None].astype(np.float64) * 0.02
    m = elements.element_mass(8, Xe, 1000.0)[0]
    V = 0.02 ** 3
    for a, b in itertools.product(range(8), range(8)):
        same = int(np.sum(synth.HEX_CORNERS[a] == synth.HEX_CORNERS[b]))
        ref = 1000.0 * V / 216.0 * {3: 8, 2: 4, 1: 2, 0: 1}[same]
        assert abs(m[a, b] - ref) <= 1e-15


# ------------------------------------------------------------- patch test

@pytest.mark.parametrize("etype", [4, 8])
@pytest.mark.parametrize("mat", MATS)
def test_patch_test_interior_forces_vanish(etype, mat):
    """A homogeneous deformation q = F0 X gives zero net force at interior nodes."""
    dims = (3, 3, 3)
    if etype == 4:
        X, conn = synth.tet_block(*dims, jitter=0.2, seed=7)
    else:
        X = synth.jitter_interior(synth.grid_nodes(*dims, 0.01), *dims, 0.01, 0.2, 7)
        conn = synth.hex_connectivity(*dims)
    F0 = np.array([[1.1, 0.05, -0.02], [0.03, 0.92, 0.04], [-0.01, 0.06, 1.15]])
    q = (X @ F0.T).reshape(-1)
    E = np.full(conn.shape[0], 4000.0)
    f, _ = elements.element_matrices(etype, X, conn, q, E, 0.4, mat)
    fg = assembly.assemble_vector(X.size, conn, f).reshape(-1, 3)
    interior = ~synth.boundary_node_mask(*dims)
    assert np.abs(fg[interior]).max() <= 1e-10 * np.abs(fg).max()
    assert np.abs(fg.sum(axis=0)).max() <= 1e-10 * np.abs(fg).max()


# ------------------------------------------------------------- uniaxial bar

def _end_face_loads(X, conn, etype, Lz, T):
    """Consistent nodal loads of a uniform nominal traction T e_z on z = Lz."""
    faces = ([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]] if etype == 4 else
             [[0, 1, 2, 3], [4, 5, 6, 7], [0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [3, 0, 4, 7]])
    loads = np.zeros(X.shape)
    for e in range(conn.shape[0]):
        for fc in faces:
            nodes = conn[e, fc]
            if np.all(np.abs(X[nodes, 2] - Lz) < 1e-12):
                P = X[nodes]
                if len(nodes) == 3:
                    area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
                else:
                    area = np.linalg.norm(np.cross(P[1] - P[0], P[3] - P[0]))
                loads[nodes, 2] += T * area / len(nodes)
    return loads


def _nh_lateral(a, mu, lam):
    """Root b of mu (b^2 - 1) + lam ln(a b^2) = 0 by bisection."""
    lo, hi = 0.2, 1.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mu * (mid * mid - 1) + lam * np.log(a * mid * mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("etype", [4, 8])
@pytest.mark.parametrize("mat", MATS)
def test_uniaxial_bar_closed_form(etype, mat):
    """Roller-supported bar under end traction reaches the exact homogeneous
    stretch: StVK T = E a (a^2 - 1)/2, b^2 = 1 - nu (a^2 - 1); NH
    T = mu (a^2 - b^2)/a with mu (b^2 - 1) + lam ln(a b^2) = 0.  The
    equilibrium is the fixed point of the step with v reset (b = p - f)."""
    dims = (2, 2, 3)
    sp = 0.01
    E0, nu = 4000.0, 0.35
    if etype == 4:
        X, conn = synth.tet_block(*dims, spacing=sp, jitter=0.2, seed=11)
    else:
        X, conn = synth.hex_beam(*dims, spacing=sp)
    Lz = dims[2] * sp
    a = 1.15
    mu, lam = elements.lame(E0, nu)
    if mat == elements.ST_VENANT_KIRCHHOFF:
        b = np.sqrt(1 - nu * (a * a - 1))
        T = E0 * a * (a * a - 1) / 2
    else:
        b = _nh_lateral(a, mu, lam)
        T = mu * (a * a - b * b) / a
    fixed = np.zeros((X.shape[0], 3), dtype=np.uint8)
    fixed[np.abs(X[:, 2]) < 1e-12, 2] = 1
    origin = np.flatnonzero(np.all(np.abs(X) < 1e-12, axis=1))[0]
    fixed[origin, :2] = 1
    xnode = np.flatnonzero((np.abs(X[:, 0] - dims[0] * sp) < 1e-12) & (np.abs(X[:, 1]) < 1e-12)
                           & (np.abs(X[:, 2]) < 1e-12))[0]
    fixed[xnode, 1] = 1
    w = synth.Workload(name="bar", elem_type=etype, X=X, conn=conn, fixed=fixed.reshape(-1),
                       E=np.full(conn.shape[0], E0), nu=nu, rho=1.0, material=mat,
                       h=1e3, alpha=0.0, beta=0.0, gravity=np.zeros(3),
                       f_nodal=_end_face_loads(X, conn, etype, Lz, T))
    pat = step.pattern(w)
    q = w.q0()
    for _ in range(30):
        q, _, _ = step.step(w, q, np.zeros_like(q), solver="dense", pat=pat)
    expect = (X * np.array([b, b, a])).reshape(-1)
    assert np.abs(q - expect).max() <= 1e-9 * Lz


# ------------------------------------------------------------- free fall

@pytest.mark.parametrize("mesh", MESHES)
def test_free_fall_scalar_recurrence(mesh):
    """No BCs, gravity, from rest: v_n = c_n g with
    c_{n+1} = c_n + h (1 - alpha c_n) / (1 + h alpha)."""
    w = synth.make(mesh)
    w.fixed = np.zeros_like(w.fixed)
    states = step.rollout(w, w.q0(), w.v0(), 4)
    c = 0.0
    for n in range(1, 5):
        c = c + w.h * (1 - w.alpha * c) / (1 + w.h * w.alpha)
        v = states[n][1].reshape(-1, 3)
        assert np.abs(v - c * w.gravity).max() <= 1e-12 * np.abs(w.gravity).max()


# ------------------------------------------------------------- pattern

def _closed_form_node_blocks(w):
    n = np.asarray(w.dims) + 1
    if w.elem_type == 8:
        return int(np.prod(3 * n - 2))
    N = int(np.prod(n))
    tot = 0
    for d in itertools.product((0, 1), repeat=3):
        if d != (0, 0, 0):
            tot += int(np.prod(n - np.asarray(d)))
    # only the Kuhn main-diagonal family of offsets is connected: (1,0,0),
    # (0,1,0), (0,0,1), (1,1,0), (0,1,1), (1,0,1), (1,1,1) and their negatives
    return N + 2 * tot


@pytest.mark.parametrize("mesh", ["tiny_tet", "tiny_hex", "tet_beam", "hex_diff"])
def test_pattern_counts_closed_form(mesh):
    w = synth.make(mesh)
    w.fixed = np.zeros_like(w.fixed)
    p = step.pattern(w)
    assert p.nnz == 9 * _closed_form_node_blocks(w)
    # structural symmetry and sorted, duplicate-free columns
    rows = np.repeat(np.arange(p.n), np.diff(p.row_ptr))
    A = set(zip(rows.tolist(), p.col_idx.tolist()))
    assert all((c, r) in A for r, c in A)
    for i in range(p.n):
        seg = p.col_idx[p.row_ptr[i]:p.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)
    per_row = np.diff(p.row_ptr)
    assert per_row.max() == (81 if w.elem_type == 8 else 45)


def test_pattern_map_brute_force():
    """Map and pattern vs a dictionary-based brute force on a tiny mesh."""
    w = synth.make("tiny_tet")
    p = step.pattern(w)
    rows, cols = assembly.triplet_keys(w.conn)
    fixed = w.fixed.astype(bool)
    keys = sorted({(r, c) for r, c in zip(rows.tolist(), cols.tolist())
                   if not fixed[r] and not fixed[c]} | {(d, d) for d in np.flatnonzero(fixed)})
    pos = {k: i for i, k in enumerate(keys)}
    assert p.nnz == len(keys)
    assert [c for _, c in keys] == p.col_idx.tolist()
    for t, (r, c) in enumerate(zip(rows.tolist(), cols.tolist())):
        expect = -1 if (fixed[r] or fixed[c]) else pos[(r, c)]
        assert p.tmap[t] == expect
    for d in np.flatnonzero(fixed):
        seg = p.col_idx[p.row_ptr[d]:p.row_ptr[d + 1]]
        assert seg.tolist() == [d]


# ------------------------------------------------------------- solves, step

def test_solvers_agree_and_residual_certified():
    w = synth.make("tet_beam")
    q, v = step.rollout(w, w.q0(), w.v0(), 3)[-1]
    s = step.assemble(w, q, v)
    p = s.pat
    xd = solve.dense_cholesky_solve(p.n, p.row_ptr, p.col_idx, s.vals, s.b)
    xb = solve.banded_cholesky_solve(p.n, p.row_ptr, p.col_idx, s.vals, s.b)
    xp, it, res = solve.jacobi_pcg(p.row_ptr, p.col_idx, s.vals, s.b, 1e-12)
    r = s.b - assembly.csr_matvec(p.row_ptr, p.col_idx, s.vals, xd)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(s.b)
    assert np.abs(xb - xd).max() <= 1e-10 * np.abs(xd).max()
    assert res <= 1e-12 and np.abs(xp - xd).max() <= 1e-8 * np.abs(xd).max()
    A = assembly.csr_to_dense(p.n, p.row_ptr, p.col_idx, s.vals)
    assert np.allclose(A, A.T, rtol=0, atol=1e-13 * np.abs(A).max())
    np.linalg.cholesky(A)                       # A is SPD near rest


def test_step_system_matches_dense_definition():
    """A and b from the triplet assembly equal the dense sums of the global
    M, K and forces built element by element (brute force)."""
    w = synth.make("tiny_hex", material=elements.ST_VENANT_KIRCHHOFF)
    q, v = synth.random_state(w, 0.1, 4)
    s = step.assemble(w, q, v)
    n = w.n_dofs
    f, K = elements.element_matrices(w.elem_type, w.X, w.conn, q, w.E, w.nu, w.material)
    m = elements.element_mass(w.elem_type, w.X[w.conn], w.rho)
    Kg = np.zeros((n, n)); Mg = np.zeros((n, n)); fg = np.zeros(n)
    for e in range(w.n_elems):
        dofs = (3 * w.conn[e][:, None] + np.arange(3)).reshape(-1)
        Kg[np.ix_(dofs, dofs)] += K[e]
        Mg[np.ix_(dofs, dofs)] += np.kron(m[e], np.eye(3))
        fg[dofs] += f[e].reshape(-1)
    p = Mg @ np.tile(w.gravity, w.n_nodes) + w.f_nodal.reshape(-1)
    A = (1 + w.h * w.alpha) * Mg + w.h * (w.beta + w.h) * Kg
    b = p - fg - w.alpha * Mg @ v - (w.beta + w.h) * Kg @ v
    fixed = w.fixed.astype(bool)
    A[fixed, :] = 0.0; A[:, fixed] = 0.0
    A[fixed, fixed] = 1.0
    b[fixed] = 0.0
    Ao = assembly.csr_to_dense(n, s.pat.row_ptr, s.pat.col_idx, s.vals)
    assert np.abs(Ao - A).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(s.b - b).max() <= 1e-13 * np.abs(b).max()


# ------------------------------------------------------------- adjoint

@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_adjoint_matches_complex_step_rollout(mesh, mat):
    """The adjoint recursion vs complex-step derivatives of the full forward
    rollout (exact to roundoff), for dL/dE_e, dL/dq0 and dL/dv0."""
    w = synth.make(mesh, material=mat)
    nsteps = 3
    E = synth.lognormal_E(w.n_elems, 5000.0, 0.3, 0)
    q0, v0 = synth.random_state(w, 0.05, 1)
    states = step.rollout(w, q0, v0, nsteps, E)
    target = states[-1][0] + 1e-4 * synth.random_vector(w.n_dofs, 3)
    dE, dq0, dv0 = adjoint.adjoint_rollout(w, E, states, 2 * (states[-1][0] - target),
                                           np.zeros(w.n_dofs))
    rng = np.random.default_rng(4)
    for k in rng.choice(w.n_elems, 3, replace=False):
        e = np.zeros(w.n_elems); e[k] = 1.0
        cs = adjoint.rollout_loss_complex_step(w, E, q0, v0, target, nsteps, dE=e)
        assert abs(dE[k] - cs) <= 1e-9 * max(abs(cs), 1e-3 * np.abs(dE).max())
    d = synth.random_vector(w.n_dofs, 6)
    cs = adjoint.rollout_loss_complex_step(w, E, q0, v0, target, nsteps, dq0=d)
    assert abs(dq0 @ d - cs) <= 1e-9 * abs(cs)
    cs = adjoint.rollout_loss_complex_step(w, E, q0, v0, target, nsteps, dv0=d)
    assert abs(dv0 @ d - cs) <= 1e-9 * abs(cs)


def test_third_derivative_symmetry():
    """T(q)[mu, w] . z is symmetric in (mu, w, z): third derivative of energy."""
    w = synth.make("tiny_hex")
    q = _deformed(w)
    rng = np.random.default_rng(8)
    a, b, c = (rng.standard_normal(w.n_dofs) * 1e-3 for _ in range(3))
    t1 = adjoint.third_derivative(w, q, w.E, a, b) @ c
    t2 = adjoint.third_derivative(w, q, w.E, c, a) @ b
    t3 = adjoint.third_derivative(w, q, w.E, b, c) @ a
    assert abs(t1 - t2) <= 1e-10 * abs(t1) and abs(t1 - t3) <= 1e-10 * abs(t1)


@pytest.mark.parametrize("mesh", MESHES)
@pytest.mark.parametrize("mat", MATS)
def test_linearised_step_is_consistent_with_backward_euler(mesh, mat):
    """A and b are the first-order Taylor linearisation of the implicit
    residual R(a) = M a - p + f(q + h v + h^2 a) + B (v + h a), B = alpha M +
    beta K(q).  Built here from the oracle's f only (no K formula):
    b - (-R(0)) = O(h^2) and A d - dR/da d = O(h^3), so halving h divides the
    mismatches by ~4 and ~8; a wrong sign or coefficient breaks the ratios."""
    w0 = synth.make(mesh, material=mat)
    q, v = synth.random_state(w0, 0.003, 3)
    v = v * 0.2
    nen = w0.conn.shape[1]
    rng = np.random.default_rng(12)
    dirn = rng.standard_normal(w0.n_dofs) * (1 - w0.fixed)
    free = ~w0.fixed.astype(bool)
    mism_b, mism_A = [], []
    for h in (0.02, 0.01):
        w = synth.make(mesh, material=mat)
        w.h = h
        s = step.assemble(w, q, v)

        def fglob(qq):
            f, _ = elements.element_matrices(w.elem_type, w.X, w.conn, qq, w.E, w.nu, mat)
            return assembly.assemble_vector(w.n_dofs, w.conn, f)

        ed = s.ed
        Mv = assembly.assemble_vector(w.n_dofs, w.conn, np.einsum(
            "eij,ej->ei", ed.M, v.reshape(-1, 3)[w.conn].reshape(-1, 3 * nen)).reshape(-1, nen, 3))
        p = assembly.assemble_vector(w.n_dofs, w.conn, ed.p_grav) + w.f_nodal.reshape(-1)
        # beta K v by central difference of f along v (K from f only)
        eps = 1e-6
        Kv = (fglob(q + eps * v) - fglob(q - eps * v)) / (2 * eps)
        negR0 = p - fglob(q + h * v) - w.alpha * Mv - w.beta * Kv
        mism_b.append(np.linalg.norm((s.b - negR0)[free]))

        def R(a):
            Ma = assembly.assemble_vector(w.n_dofs, w.conn, np.einsum(
                "eij,ej->ei", ed.M, a.reshape(-1, 3)[w.conn].reshape(-1, 3 * nen)).reshape(-1, nen, 3))
            Ka = (fglob(q + eps * a) - fglob(q - eps * a)) / (2 * eps)
            return Ma - p + fglob(q + h * v + h * h * a) + w.alpha * (Mv + h * Ma) + w.beta * (Kv + h * Ka)

        dR = (R(1e-3 * dirn) - R(-1e-3 * dirn)) / 2e-3
        Ad = assembly.csr_matvec(s.pat.row_ptr, s.pat.col_idx, s.vals, dirn)
        mism_A.append(np.linalg.norm((Ad - dR)[free]))
        rel_A = mism_A[-1] / np.linalg.norm(dR[free])
    assert 3.0 < mism_b[0] / mism_b[1] < 5.0
    assert rel_A < 1e-2
    assert 6.0 < mism_A[0] / mism_A[1] < 10.0
