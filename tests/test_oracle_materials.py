"""Pins of the oracle's Mooney-Rivlin and co-rotational elements (paper Sec.
3.1: co-rotational elements and MJED hyperelastic materials) against facts
that do not come from the oracle's own formulas: complex-step derivatives of
the energy and of the element force, the closed forms of linear elasticity at
rest and of pure dilation, rigid motions, rotation covariance and the
defining properties of a polar decomposition."""
import numpy as np
import pytest

import synth
from oracle import elements as el

MU, LAM, SHARE = 1200.0, 3000.0, 0.3
MR, CR = el.MOONEY_RIVLIN, el.COROTATIONAL


def _rand_F(rng, n, scale=0.3):
    F = np.eye(3) + scale * rng.uniform(-1, 1, size=(n, 3, 3))
    assert np.all(np.linalg.det(F) > 0.2)
    return F


def _rot(rng):
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def test_mooney_rivlin_stress_is_energy_gradient():
    rng = np.random.default_rng(0)
    F = _rand_F(rng, 6)
    P = el.first_piola(F, MU, LAM, MR, SHARE)
    h = 1e-30
    for k in range(3):
        for l in range(3):
            Fc = F.astype(np.complex128)
            Fc[:, k, l] += 1j * h
            dpsi = el.energy_density(Fc, MU, LAM, MR, SHARE).imag / h
            assert np.allclose(dpsi, P[:, k, l], rtol=1e-12, atol=1e-9 * MU)


def test_mooney_rivlin_rest_is_linear_elasticity():
    A = el.elasticity_tensor(np.eye(3)[None], MU, LAM, MR, SHARE)[0]
    d = np.eye(3)
    lin = (LAM * np.einsum("ij,kl->ijkl", d, d)
           + MU * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    assert np.abs(A - lin).max() <= 1e-9 * MU
    assert np.abs(el.first_piola(np.eye(3)[None], MU, LAM, MR, SHARE)).max() <= 1e-12 * MU


def test_mooney_rivlin_pure_dilation_closed_form():
    # F = s I: the isochoric invariants stay 3, Psi = kappa/2 (3 ln s)^2,
    # P = kappa (3 ln s) / s I
    kappa = LAM + 2.0 * MU / 3.0
    for s in (0.8, 1.0, 1.3):
        F = s * np.eye(3)[None]
        assert abs(el.energy_density(F, MU, LAM, MR, SHARE)[0]
                   - 0.5 * kappa * (3 * np.log(s)) ** 2) <= 1e-9 * kappa
        P = el.first_piola(F, MU, LAM, MR, SHARE)[0]
        assert np.abs(P - kappa * 3 * np.log(s) / s * np.eye(3)).max() <= 1e-9 * kappa


def test_mooney_rivlin_objectivity_and_major_symmetry():
    rng = np.random.default_rng(1)
    F = _rand_F(rng, 5)
    Q = _rot(rng)
    QF = np.einsum("ij,ejk->eik", Q, F)
    assert np.allclose(el.energy_density(QF, MU, LAM, MR, SHARE),
                       el.energy_density(F, MU, LAM, MR, SHARE), rtol=1e-12)
    assert np.allclose(el.first_piola(QF, MU, LAM, MR, SHARE),
                       np.einsum("ij,ejk->eik", Q, el.first_piola(F, MU, LAM, MR, SHARE)),
                       rtol=1e-10, atol=1e-9 * MU)
    A = el.elasticity_tensor(F, MU, LAM, MR, SHARE)
    assert np.abs(A - np.einsum("eijkl->eklij", A)).max() <= 1e-8 * MU


@pytest.mark.parametrize("name", ["tiny_tet", "tiny_hex"])
def test_mooney_rivlin_element_stiffness_is_force_derivative(name):
    # K from the elasticity tensor and the shape gradients vs the complex
    # step of the element force with respect to each nodal coordinate
    w = synth.make(name, material=MR)
    rng = np.random.default_rng(2)
    Xe = w.X[w.conn][:3]
    xe = Xe + 0.002 * rng.uniform(-1, 1, size=Xe.shape)
    E = np.array([5000.0, 6000.0, 7000.0])
    mu, lam = el.lame(E, w.nu)
    G, dV = el.quadrature(w.elem_type, Xe)
    K = el.element_stiffness(xe, G, dV, mu, lam, MR, SHARE)
    h = 1e-30
    nen = Xe.shape[1]
    for b in range(nen):
        for j in range(3):
            xc = xe.astype(np.complex128)
            xc[:, b, j] += 1j * h
            df = el.element_force(xc, G, dV, mu, lam, MR, SHARE).imag / h
            assert np.abs(df - K[:, :, :, b, j]).max() <= 1e-9 * np.abs(K).max()
    Kf = K.reshape(3, 3 * nen, 3 * nen)
    assert np.abs(Kf - np.swapaxes(Kf, 1, 2)).max() <= 1e-9 * np.abs(Kf).max()


@pytest.mark.parametrize("name", ["tiny_tet", "tiny_hex"])
def test_corotational_rigid_motion_and_rest(name):
    w = synth.make(name, material=CR)
    rng = np.random.default_rng(3)
    Xe = w.X[w.conn]
    E = np.full(Xe.shape[0], 5000.0)
    mu, lam = el.lame(E, w.nu)
    G, dV = el.quadrature(w.elem_type, Xe)
    K0 = el.element_stiffness(Xe, G, dV, mu, lam, el.ST_VENANT_KIRCHHOFF)
    # at rest: no force, K = K0 (linear elasticity)
    f, K = el.corotational_force_stiffness(w.elem_type, Xe, Xe.copy(), mu, lam)
    assert np.abs(f).max() <= 1e-12 * np.abs(K0).max() * 0.01
    assert np.abs(K - K0).max() <= 1e-12 * np.abs(K0).max()
    # rigid motion x = Q X + t: no force, K = Q K0 Q^T blockwise
    Q = _rot(rng)
    t = rng.uniform(-1, 1, 3)
    xe = np.einsum("ij,eaj->eai", Q, Xe) + t
    f, K = el.corotational_force_stiffness(w.elem_type, Xe, xe, mu, lam)
    assert np.abs(f).max() <= 1e-10 * np.abs(K0).max() * 0.01
    assert np.abs(K - np.einsum("ij,eajbk,lk->eaibl", Q, K0, Q)).max() <= 1e-10 * np.abs(K0).max()


@pytest.mark.parametrize("name", ["tiny_tet", "tiny_hex"])
def test_corotational_covariance_and_small_strain(name):
    w = synth.make(name, material=CR)
    rng = np.random.default_rng(4)
    Xe = w.X[w.conn]
    E = np.full(Xe.shape[0], 5000.0)
    mu, lam = el.lame(E, w.nu)
    G, dV = el.quadrature(w.elem_type, Xe)
    K0 = el.element_stiffness(Xe, G, dV, mu, lam, el.ST_VENANT_KIRCHHOFF)
    u = rng.uniform(-1, 1, size=Xe.shape)
    xe = Xe + 0.002 * u
    f, K = el.corotational_force_stiffness(w.elem_type, Xe, xe, mu, lam)
    # rotating the deformed element rotates force and stiffness
    Q = _rot(rng)
    fq, Kq = el.corotational_force_stiffness(w.elem_type, Xe, np.einsum("ij,eaj->eai", Q, xe),
                                             mu, lam)
    assert np.abs(fq - np.einsum("ij,eaj->eai", Q, f)).max() <= 1e-9 * np.abs(f).max()
    assert np.abs(Kq - np.einsum("ij,eajbk,lk->eaibl", Q, K, Q)).max() <= 1e-9 * np.abs(K).max()
    # small strain: f = K0 u to second order in the displacement
    errs = []
    for s in (1e-3, 5e-4):
        fs, _ = el.corotational_force_stiffness(w.elem_type, Xe, Xe + s * u, mu, lam)
        lin = np.einsum("eaibj,ebj->eai", K0, s * u)
        errs.append(np.abs(fs - lin).max())
    assert errs[1] / errs[0] < 0.3          # second order: ratio 1/4
    # K symmetric
    nen = Xe.shape[1]
    Kf = K.reshape(-1, 3 * nen, 3 * nen)
    assert np.abs(Kf - np.swapaxes(Kf, 1, 2)).max() <= 1e-12 * np.abs(Kf).max()


def test_corotational_rotation_is_polar_factor():
    w = synth.make("tiny_hex", material=CR)
    rng = np.random.default_rng(5)
    Xe = w.X[w.conn]
    Q = _rot(rng)
    xe = np.einsum("ij,eaj->eai", Q, Xe + 0.003 * rng.uniform(-1, 1, size=Xe.shape))
    R = el.corotational_rotation(w.elem_type, Xe, xe)
    Fc = np.einsum("eai,eaj->eij", xe, el.centre_gradients(w.elem_type, Xe))
    assert np.abs(np.einsum("eji,ejk->eik", R, R) - np.eye(3)).max() <= 1e-13
    assert np.all(np.abs(np.linalg.det(R) - 1.0) <= 1e-13)
    U = np.einsum("eji,ejk->eik", R, Fc)
    assert np.abs(U - np.swapaxes(U, 1, 2)).max() <= 1e-13
    assert np.all(np.linalg.eigvalsh(0.5 * (U + np.swapaxes(U, 1, 2))) > 0)
    # the centre gradients reproduce an affine field exactly
    B = rng.uniform(-1, 1, (3, 3))
    Fa = np.einsum("eai,eaj->eij", np.einsum("ij,eaj->eai", B, Xe),
                   el.centre_gradients(w.elem_type, Xe))
    assert np.abs(Fa - B).max() <= 1e-12
