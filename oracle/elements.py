"""Per-element quantities (FP64 or complex128), oracle side.

The paper (Sec. 3.1) uses co-rotational elements (element stiffness from the
strain-displacement and stress-strain matrices, Eq. "eqmodel") and MJED
hyperelastic elements (Mooney-Rivlin, St Venant-Kirchhoff), written in the
invariants I1 = tr C, I2 = ((tr C)^2 - tr C^2)/2 and J = det F, and prints no
further formulas.  The laws below are textbook forms (readings R4, R22, R23
of the design notes):

* neo-Hookean (Bonet & Wood), St Venant-Kirchhoff: P = dPsi/dF, K = the exact
  Hessian of the stored energy;
* Mooney-Rivlin, decoupled compressible form in the isochoric invariants
  J^{-2/3} I1, J^{-4/3} I2 plus kappa/2 (ln J)^2; K = the exact Hessian, with
  the elasticity tensor dP/dF taken by complex step of P;
* co-rotational: the element rotation R is the rotation factor of the polar
  decomposition of F at the element centre; f = R K0 (R^T x - X) and
  K = R K0 R^T with K0 the small-strain (linear elastic) element stiffness;
  K holds R fixed, as co-rotational elements do, so it is not df/dx.

Sec. 3.2 writes M a = p - F(q, v); K enters A as the stiffness of F.

All arrays carry a leading element axis.  The neo-Hookean and St
Venant-Kirchhoff functions accept complex input, so that complex-step
derivatives can be taken through them.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# material constants


def lame(E, nu):
    """Lame parameters (mu, lambda) from Young's modulus and Poisson ratio."""
    E = np.asarray(E)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


# --------------------------------------------------------------------------
# reference-configuration shape gradients

HEX_SIGNS = np.array(
    [[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
GAUSS_1D = np.array([-1.0, 1.0]) / np.sqrt(3.0)


def hex_gauss_points():
    """The 2x2x2 Gauss points (xi, eta, zeta) with unit weights, [8, 3]."""
    pts = np.array([[x, y, z] for z in GAUSS_1D for y in GAUSS_1D for x in GAUSS_1D])
    return pts, np.ones(8)


def hex_shape(xi):
    """Trilinear shape values N_a(xi) [Q, 8] and derivatives dN_a/dxi [Q, 8, 3]."""
    xi = np.atleast_2d(xi)
    t = 1.0 + HEX_SIGNS[None, :, :] * xi[:, None, :]          # [Q, 8, 3]
    N = 0.125 * t.prod(axis=2)
    dN = np.empty(t.shape)
    for i in range(3):
        others = [j for j in range(3) if j != i]
        dN[:, :, i] = 0.125 * HEX_SIGNS[None, :, i] * t[:, :, others[0]] * t[:, :, others[1]]
    return N, dN


def tet_gradients(Xe):
    """TET4: gradients g_a = grad_X N_a [E, 4, 3] and volume V [E].

    With D_m = [X1-X0, X2-X0, X3-X0] (columns), the map X(s) = X0 + D_m s is
    linear, so grad_X N_a for a = 1..3 is row a-1 of D_m^{-1} and
    g_0 = -(g_1 + g_2 + g_3).
    """
    Dm = np.transpose(Xe[:, 1:, :] - Xe[:, :1, :], (0, 2, 1))
    Dinv = np.linalg.inv(Dm)
    g = np.empty(Xe.shape, dtype=Dinv.dtype)
    g[:, 1:, :] = Dinv
    g[:, 0, :] = -Dinv.sum(axis=1)
    V = np.abs(np.linalg.det(Dm)) / 6.0
    return g, V


def hex_gradients(Xe):
    """HEX8: per Gauss point gradients G [E, 8gp, 8, 3] and dV = w det J [E, 8gp].

    J = sum_a X_a (x) dN_a/dxi, g_a = J^{-T} dN_a/dxi.
    """
    pts, wts = hex_gauss_points()
    _, dN = hex_shape(pts)                                   # [Q, 8, 3]
    J = np.einsum("eai,qaj->eqij", Xe, dN)                   # [E, Q, 3, 3]
    Jinv = np.linalg.inv(J)
    G = np.einsum("qaj,eqji->eqai", dN, Jinv)                # g_a,i = sum_j dN_a,j Jinv_ji
    detJ = np.linalg.det(J)
    return G, detJ * wts[None, :]


def quadrature(elem_type, Xe):
    """Uniform interface: (G [E, Q, nen, 3], dV [E, Q])."""
    if elem_type == 4:
        g, V = tet_gradients(Xe)
        return g[:, None, :, :], V[:, None]
    if elem_type == 8:
        return hex_gradients(Xe)
    raise ValueError(elem_type)


# --------------------------------------------------------------------------
# material laws (per quadrature point; F has shape [..., 3, 3])

NEO_HOOKEAN = 0
ST_VENANT_KIRCHHOFF = 1
COROTATIONAL = 2
MOONEY_RIVLIN = 3


def mooney_rivlin_constants(mu, lam, share):
    """(C10, C01, kappa): C10 + C01 = mu / 2 split by `share` (the part of
    C01), kappa = lam + 2 mu / 3, so that the small-strain limit is linear
    elasticity with the same (mu, lambda)."""
    mu = np.asarray(mu)
    return (1.0 - share) * 0.5 * mu, share * 0.5 * mu, np.asarray(lam) + 2.0 * mu / 3.0


def _inv_T(F):
    return np.swapaxes(np.linalg.inv(F), -1, -2)


def _invariants(F):
    C = np.swapaxes(F, -1, -2) @ F
    I1 = np.trace(C, axis1=-2, axis2=-1)
    I2 = 0.5 * (I1 ** 2 - np.einsum("...ij,...ji->...", C, C))
    J = np.linalg.det(F)
    return C, I1, I2, J


def energy_density(F, mu, lam, material, share=0.25):
    """Stored energy per unit reference volume."""
    if material == MOONEY_RIVLIN:
        c10, c01, kappa = mooney_rivlin_constants(mu, lam, share)
        _, I1, I2, J = _invariants(F)
        lnJ = np.log(J)
        return (c10 * (J ** (-2.0 / 3.0) * I1 - 3.0) + c01 * (J ** (-4.0 / 3.0) * I2 - 3.0)
                + 0.5 * kappa * lnJ ** 2)
    if material == NEO_HOOKEAN:
        J = np.linalg.det(F)
        lnJ = np.log(J)
        I1 = np.einsum("...ij,...ij->...", F, F)
        return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2
    if material == ST_VENANT_KIRCHHOFF:
        Eg = 0.5 * (np.swapaxes(F, -1, -2) @ F - np.eye(3))
        tr = np.trace(Eg, axis1=-2, axis2=-1)
        return 0.5 * lam * tr ** 2 + mu * np.einsum("...ij,...ij->...", Eg, Eg)
    raise ValueError(material)


def first_piola(F, mu, lam, material, share=0.25):
    """First Piola-Kirchhoff stress P = dPsi/dF."""
    mu = np.asarray(mu)[..., None, None]
    lam = np.asarray(lam)[..., None, None]
    if material == MOONEY_RIVLIN:
        # dI1/dF = 2F, dI2/dF = 2(I1 F - F C), dJ/dF = J F^{-T}
        c10, c01, kappa = mooney_rivlin_constants(mu, lam, share)
        C, I1, I2, J = _invariants(F)
        FiT = _inv_T(F)
        I1, I2, J = I1[..., None, None], I2[..., None, None], J[..., None, None]
        return (2.0 * c10 * J ** (-2.0 / 3.0) * (F - I1 / 3.0 * FiT)
                + 2.0 * c01 * J ** (-4.0 / 3.0) * (I1 * F - F @ C - 2.0 / 3.0 * I2 * FiT)
                + kappa * np.log(J) * FiT)
    if material == NEO_HOOKEAN:
        FiT = _inv_T(F)
        lnJ = np.log(np.linalg.det(F))[..., None, None]
        return mu * (F - FiT) + lam * lnJ * FiT
    if material == ST_VENANT_KIRCHHOFF:
        Eg = 0.5 * (np.swapaxes(F, -1, -2) @ F - np.eye(3))
        S = lam * np.trace(Eg, axis1=-2, axis2=-1)[..., None, None] * np.eye(3) + 2.0 * mu * Eg
        return F @ S
    raise ValueError(material)


def deformation_gradient(xe, G):
    """F = sum_a x_a (x) g_a at each quadrature point: [E, Q, 3, 3]."""
    return np.einsum("eai,eqaj->eqij", xe, G)


def elasticity_tensor(F, mu, lam, material, share=0.25):
    """A[..., i, j, k, l] = dP_ij / dF_kl by complex step of P (exact to
    rounding; F real)."""
    F = np.asarray(F, dtype=np.float64)
    step = 1e-30
    A = np.empty(F.shape + (3, 3))
    for k in range(3):
        for l in range(3):
            Fc = F.astype(np.complex128)
            Fc[..., k, l] += 1j * step
            A[..., k, l] = first_piola(Fc, mu, lam, material, share).imag / step
    return A


def centre_gradients(elem_type, Xe):
    """Shape gradients g_a at the element centre, [E, nen, 3] (TET4: the
    constant gradients; HEX8: xi = 0)."""
    if elem_type == 4:
        g, _ = tet_gradients(Xe)
        return g
    _, dN = hex_shape(np.zeros((1, 3)))
    J = np.einsum("eai,aj->eij", Xe, dN[0])
    return np.einsum("aj,eji->eai", dN[0], np.linalg.inv(J))


def corotational_rotation(elem_type, Xe, xe):
    """Rotation factor R of the polar decomposition F_c = R U of the
    deformation gradient at the element centre, [E, 3, 3]."""
    import scipy.linalg as sla
    Fc = np.einsum("eai,eaj->eij", xe, centre_gradients(elem_type, Xe))
    return np.stack([sla.polar(F)[0] for F in Fc])


def corotational_force_stiffness(elem_type, Xe, xe, mu, lam):
    """Co-rotational element: f_a = R sum_b K0_ab (R^T x_b - X_b) and
    K_ab = R K0_ab R^T, positions relative to node 0 (K0 annihilates
    translations).  Returns f [E, nen, 3] and K [E, nen, 3, nen, 3]."""
    G, dV = quadrature(elem_type, Xe)
    K0 = element_stiffness(Xe, G, dV, mu, lam, ST_VENANT_KIRCHHOFF)   # at rest: linear elastic
    R = corotational_rotation(elem_type, Xe, xe)
    d = np.einsum("eji,eaj->eai", R, xe - xe[:, :1]) - (Xe - Xe[:, :1])
    f = np.einsum("eij,eajbk,ebk->eai", R, K0, d)
    K = np.einsum("eij,eajbk,elk->eaibl", R, K0, R)
    return f, K


# --------------------------------------------------------------------------
# element quantities


def element_energy(xe, G, dV, mu, lam, material):
    F = deformation_gradient(xe, G)
    psi = energy_density(F, mu[:, None], lam[:, None], material)
    return np.sum(psi * dV, axis=1)


def element_force(xe, G, dV, mu, lam, material, share=0.25):
    """Internal (restoring) force f_a = sum_q dV P g_a, [E, nen, 3]
    (hyperelastic materials; co-rotational: corotational_force_stiffness)."""
    F = deformation_gradient(xe, G)
    P = first_piola(F, mu[:, None], lam[:, None], material, share)
    return np.einsum("eq,eqij,eqaj->eai", dV, P, G)


def element_stiffness(xe, G, dV, mu, lam, material, share=0.25):
    """Tangent K[e, a, i, b, j] = d f_{a,i} / d x_{b,j} (exact Hessian blocks).

    Mooney-Rivlin: K_ab,ik = sum_q dV g_a,j A_ijkl g_b,l with the elasticity
    tensor A = dP/dF.

    neo-Hookean, h_a = F^{-T} g_a:
        K_ab = mu (g_a.g_b) I + lam h_a h_b^T + (mu - lam ln J) h_b h_a^T
    St Venant-Kirchhoff, S = lam tr(E) I + 2 mu E:
        K_ab = (g_a^T S g_b) I + lam (F g_a)(F g_b)^T + mu (F g_b)(F g_a)^T
               + mu (g_a.g_b) F F^T
    """
    F = deformation_gradient(xe, G)
    gg = np.einsum("eqai,eqbi->eqab", G, G)
    I3 = np.eye(3)
    m = mu[:, None]
    l = lam[:, None]
    if material == MOONEY_RIVLIN:
        A = elasticity_tensor(F, m, l, material, share)
        return np.einsum("eq,eqaj,eqijkl,eqbl->eaibk", dV, G, A, G)
    if material == NEO_HOOKEAN:
        FiT = _inv_T(F)
        lnJ = np.log(np.linalg.det(F))
        H = np.einsum("eqij,eqaj->eqai", FiT, G)              # h_a
        K = (m[..., None, None, None, None] * np.einsum("eqab,ij->eqaibj", gg, I3)
             + l[..., None, None, None, None] * np.einsum("eqai,eqbj->eqaibj", H, H)
             + (m - l * lnJ)[..., None, None, None, None]
             * np.einsum("eqbi,eqaj->eqaibj", H, H))
    elif material == ST_VENANT_KIRCHHOFF:
        Eg = 0.5 * (np.swapaxes(F, -1, -2) @ F - I3)
        S = (l * np.trace(Eg, axis1=-2, axis2=-1))[..., None, None] * I3 + 2.0 * m[..., None, None] * Eg
        FG = np.einsum("eqij,eqaj->eqai", F, G)               # F g_a
        gSg = np.einsum("eqai,eqij,eqbj->eqab", G, S, G)
        FFt = F @ np.swapaxes(F, -1, -2)
        K = (np.einsum("eqab,ij->eqaibj", gSg, I3)
             + l[..., None, None, None, None] * np.einsum("eqai,eqbj->eqaibj", FG, FG)
             + m[..., None, None, None, None] * np.einsum("eqbi,eqaj->eqaibj", FG, FG)
             + m[..., None, None, None, None] * np.einsum("eqab,eqij->eqaibj", gg, FFt))
    else:
        raise ValueError(material)
    return np.einsum("eq,eqaibj->eaibj", dV, K)


def element_mass(elem_type, Xe, rho):
    """Consistent mass M[e, a, b] (the 3x3 block is M_ab I).

    TET4: M_ab = rho V (1 + delta_ab) / 20 (exact for linear shape functions).
    HEX8: M_ab = sum_q rho N_a N_b w det J (2x2x2 Gauss, exact on
    parallelepipeds).
    """
    if elem_type == 4:
        _, V = tet_gradients(Xe)
        base = (np.ones((4, 4)) + np.eye(4)) / 20.0
        return rho * V[:, None, None] * base[None]
    if elem_type == 8:
        pts, _ = hex_gauss_points()
        N, _ = hex_shape(pts)
        _, dV = hex_gradients(Xe)
        return rho * np.einsum("qa,qb,eq->eab", N, N, dV)
    raise ValueError(elem_type)


def element_force_stiffness(elem_type, Xe, xe, E, nu, material, share=0.25):
    """(f_e [E, nen, 3], K_e [E, nen, 3, nen, 3]) for any material."""
    mu, lam = lame(E, nu)
    if material == COROTATIONAL:
        return corotational_force_stiffness(elem_type, Xe, xe, mu, lam)
    G, dV = quadrature(elem_type, Xe)
    return (element_force(xe, G, dV, mu, lam, material, share),
            element_stiffness(xe, G, dV, mu, lam, material, share))


def element_matrices(elem_type, X, conn, q, E, nu, material, share=0.25):
    """Convenience: (f_e [E, nen, 3], K_e [E, 3nen, 3nen]) at positions q."""
    f, K = element_force_stiffness(elem_type, X[conn], q.reshape(-1, 3)[conn], E, nu, material,
                                   share)
    nen = conn.shape[1]
    return f, K.reshape(-1, 3 * nen, 3 * nen)
