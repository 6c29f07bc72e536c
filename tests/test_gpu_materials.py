"""The paper's other materials on the GPU (Sec. 3.1: co-rotational elements
and MJED hyperelastic Mooney-Rivlin), against the oracle: assembled A and b
(compact map and per-DOF int32 map paths), trajectories with an exact and a
stale factor, and the error paths (adjoint restricted to the materials whose
K is the Hessian of an energy; bad Mooney-Rivlin split).

Tolerances as for the other materials: FP64 1e-12 on A and b; mixed 1e-5
(the FP32 element arithmetic; the Mooney-Rivlin stress and tangent and the
co-rotational rotation are evaluated in FP64 and rounded once)."""
import numpy as np
import pytest
import torch

import synth
from oracle import step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import FE_COROTATIONAL, FE_MOONEY_RIVLIN, FEError  # noqa: E402
from paper_2306_05893_amd.sim import FEContext, Params, StepOptions  # noqa: E402

DEV = "cuda"
MATS = [FE_COROTATIONAL, FE_MOONEY_RIVLIN]


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _params(w, E=None, share=None):
    return Params(w.h, w.alpha, w.beta, w.rho, w.nu, w.material, w.gravity,
                  w.E if E is None else E, w.f_nodal, DEV,
                  w.mr_c01_share if share is None else share)


def _ctx(w, prec):
    print(f"[materials] {w.name} elem={w.elem_type} mat={w.material} prec={prec}", flush=True)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV)
    ctx.bind()
    return ctx


@pytest.mark.parametrize("mesh", ["tiny_tet", "tiny_hex", "tet_beam", "hex_diff"])
@pytest.mark.parametrize("mat", MATS)
@pytest.mark.parametrize("prec", [0, 1])
def test_assembly_parity(mesh, mat, prec):
    w = synth.make(mesh, material=mat)
    w.mr_c01_share = 0.3
    q, v = synth.random_state(w, 0.004, 6)
    ref = step.assemble(w, q, v)
    ctx = _ctx(w, prec)
    A, b = ctx.assemble(_params(w), _t(q), _t(v))
    torch.cuda.synchronize()
    ea, eb = _rel(A.double().cpu().numpy(), ref.vals), _rel(b.cpu().numpy(), ref.b)
    print(f"  A err {ea:.3e}  b err {eb:.3e}")
    tol = 1e-12 if prec == 0 else 1e-5
    assert ea <= tol and eb <= tol
    ctx.close()


@pytest.mark.parametrize("mat", MATS)
@pytest.mark.parametrize("prec", [0, 1])
def test_assembly_parity_per_dof_constraints(mat, prec):
    """Roller constraints: the int32 map path."""
    w = synth.make("tiny_hex", material=mat)
    fixed = np.zeros(w.n_dofs, dtype=np.uint8)
    fixed[2::3][np.abs(w.X[:, 2]) < 1e-12] = 1
    fixed[0] = fixed[1] = 1
    w.fixed = fixed
    q, v = synth.random_state(w, 0.003, 2)
    ref = step.assemble(w, q, v)
    ctx = _ctx(w, prec)
    assert ctx.sizes.compact_map == 0
    A, b = ctx.assemble(_params(w), _t(q), _t(v))
    torch.cuda.synchronize()
    tol = 1e-12 if prec == 0 else 1e-5
    assert _rel(A.double().cpu().numpy(), ref.vals) <= tol
    assert _rel(b.cpu().numpy(), ref.b) <= tol
    ctx.close()


def test_rigid_rotation_gives_no_elastic_force():
    # co-rotational and Mooney-Rivlin: a rigidly rotated state at rest has
    # b = gravity only (no elastic force, v = 0)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Q *= np.sign(np.linalg.det(Q))
    for mat in MATS:
        w = synth.make("tiny_hex", material=mat)
        w.fixed = np.zeros(w.n_dofs, dtype=np.uint8)
        w.gravity = np.zeros(3)
        ctx = _ctx(w, 0)
        q = (w.X @ Q.T).reshape(-1)
        A, b = ctx.assemble(_params(w), _t(q), _t(np.zeros(w.n_dofs)))
        torch.cuda.synchronize()
        ref = step.assemble(w, w.q0(), np.zeros(w.n_dofs))
        scale = np.abs(ref.vals).max() * 1e-3
        print(f"  mat {mat}: |b| {np.abs(b.cpu().numpy()).max():.2e} (A scale {scale:.2e})")
        assert np.abs(b.cpu().numpy()).max() <= 1e-9 * scale
        ctx.close()


@pytest.mark.parametrize("mat", MATS)
@pytest.mark.parametrize("prec", [0, 1])
def test_tet_beam_trajectory(mat, prec):
    """Tet beam under gravity, 6 steps, exact factor (FP64) / factor refreshed
    every 3 steps with lag 1 (mixed), vs the oracle's dense rollout."""
    w = synth.make("tet_beam", material=mat)
    n = 6
    qo, vo = step.rollout(w, w.q0(), w.v0(), n)[-1]
    ctx = _ctx(w, prec)
    p = _params(w)
    q, v = _t(w.q0()), _t(w.v0())
    opts = (StepOptions(rel_tol=1e-11, max_it=300, refresh=1, lag=0) if prec == 0 else
            StepOptions(rel_tol=1e-8, max_it=3000, refresh=3, lag=1))
    its = []
    for _ in range(n):
        st = ctx.step(q, v, p, opts)
        assert st.solve.status == 0
        its.append(st.solve.iterations)
    torch.cuda.synchronize()
    eq = np.linalg.norm(q.cpu().numpy() - qo) / np.linalg.norm(qo - w.q0())
    ev = np.linalg.norm(v.cpu().numpy() - vo) / np.linalg.norm(vo)
    print(f"  mat {mat} prec {prec}: displacement err {eq:.2e}, velocity err {ev:.2e}, its {its}")
    tol = 1e-8 if prec == 0 else 1e-4
    assert eq <= tol and ev <= tol
    ctx.close()


def test_error_paths():
    w = synth.make("tiny_hex", material=FE_MOONEY_RIVLIN)
    ctx = _ctx(w, 0)
    with pytest.raises(FEError):
        ctx.assemble(_params(w, share=1.5), _t(w.q0()), _t(w.v0()))
    n = w.n_dofs
    z = torch.zeros(n, dtype=torch.float64, device=DEV)
    dE = torch.zeros(w.n_elems, dtype=torch.float64, device=DEV)
    for mat in MATS:
        w.material = mat
        with pytest.raises(FEError):
            ctx.step_adjoint(_t(w.q0()), z, z, z, z, z.clone(), z.clone(), dE, _params(w),
                             StepOptions(rel_tol=1e-10, max_it=100, refresh=1, lag=0))
    ctx.close()
