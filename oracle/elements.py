"""Per-element hyperelastic quantities (FP64 or complex128), oracle side.

The paper (Sec. 3.1) uses co-rotational and MJED hyperelastic elements inside
SOFA and prints no element formulas; the material laws below are the textbook
forms (compressible neo-Hookean of Bonet & Wood; St Venant-Kirchhoff), the
readings listed as R3/R4 in the design notes.  The internal force is the
gradient of the stored energy and K = df/dq is its Hessian (Sec. 3.2 writes
M a = p - F(q, v); K is the derivative of F with respect to q).

All arrays carry a leading element axis.  Functions accept complex input so
that complex-step derivatives can be taken through them.
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


def _inv_T(F):
    return np.swapaxes(np.linalg.inv(F), -1, -2)


def energy_density(F, mu, lam, material):
    """Stored energy per unit reference volume."""
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


def first_piola(F, mu, lam, material):
    """First Piola-Kirchhoff stress P = dPsi/dF."""
    mu = np.asarray(mu)[..., None, None]
    lam = np.asarray(lam)[..., None, None]
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


# --------------------------------------------------------------------------
# element quantities


def element_energy(xe, G, dV, mu, lam, material):
    F = deformation_gradient(xe, G)
    psi = energy_density(F, mu[:, None], lam[:, None], material)
    return np.sum(psi * dV, axis=1)


def element_force(xe, G, dV, mu, lam, material):
    """Internal (restoring) force f_a = sum_q dV P g_a, [E, nen, 3]."""
    F = deformation_gradient(xe, G)
    P = first_piola(F, mu[:, None], lam[:, None], material)
    return np.einsum("eq,eqij,eqaj->eai", dV, P, G)


def element_stiffness(xe, G, dV, mu, lam, material):
    """Tangent K[e, a, i, b, j] = d f_{a,i} / d x_{b,j} (exact Hessian blocks).

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


def element_matrices(elem_type, X, conn, q, E, nu, material):
    """Convenience: (f_e [E, nen, 3], K_e [E, 3nen, 3nen]) at positions q."""
    Xe = X[conn]
    xe = q.reshape(-1, 3)[conn]
    G, dV = quadrature(elem_type, Xe)
    mu, lam = lame(E, nu)
    f = element_force(xe, G, dV, mu, lam, material)
    K = element_stiffness(xe, G, dV, mu, lam, material)
    nen = conn.shape[1]
    return f, K.reshape(-1, 3 * nen, 3 * nen)
