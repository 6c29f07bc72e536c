"""GPU multifrontal refactorisation (factor_on_gpu) against the oracle.

The preconditioner built on the GPU must apply A_t0^{-1}: z = P^{-1} r is
compared with the oracle's dense / banded solve and with the host
factorisation's panels (same ordering, same explicit-inverse form).  Steps
driven with the GPU factor are compared with the oracle's trajectory.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import assembly, solve, step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import _lib  # noqa: E402
from paper_2306_05893_amd.sim import FEContext, Params, StepOptions  # noqa: E402

DEV = "cuda"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _params(w):
    return Params(w.h, w.alpha, w.beta, w.rho, w.nu, w.material, w.gravity, w.E, w.f_nodal, DEV)


@pytest.mark.parametrize("mesh", ["tiny_tet", "tiny_hex", "tet_beam", "hex_diff"])
@pytest.mark.parametrize("prec", [0, 1])
def test_gpu_factor_applies_inverse(mesh, prec):
    w = synth.make(mesh)
    print(f"[gpu-factor] {mesh} prec={prec}", flush=True)
    q, v = step.rollout(w, w.q0(), w.v0(), 2)[-1]
    ref = step.assemble(w, q, v)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV, factor_on_gpu=True)
    A, _ = ctx.assemble(_params(w), _t(q), _t(v))
    assert ctx.factorize_now(A, 3) == 3
    r = synth.random_vector(w.n_dofs, 4)
    z = ctx.precond_apply(_t(r)).cpu().numpy()
    Ag = A.double().cpu().numpy()
    p = ref.pat
    z_ref = (solve.dense_cholesky_solve if w.n_dofs < 4000 else solve.banded_cholesky_solve)(
        p.n, p.row_ptr, p.col_idx, Ag, r)
    z_host = ctx.host_factor_apply(Ag, r[None])[0]
    e1, e2 = _rel(z, z_ref), _rel(z, z_host)
    print(f"  err vs direct solve {e1:.2e}, vs host panels {e2:.2e}")
    assert e1 <= (1e-9 if prec == 0 else 1e-5)
    assert e2 <= (1e-10 if prec == 0 else 1e-5)
    ctx.close()


def test_gpu_factor_hex_beam_fp64():
    """The benchmark mesh (107,163 DOFs) in FP64: its levels use both update
    tile widths (128 for the large Schur complements, 64 for the panel steps
    and the top levels) and every panel-step path; P^{-1} r against the
    oracle's banded solve of the same matrix."""
    w = synth.make("hex_beam")
    print("[gpu-factor] hex_beam fp64 oracle assembly", flush=True)
    q, v = synth.random_state(w, 0.002, 5)
    ref = step.assemble(w, q, v)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=0, device=DEV, factor_on_gpu=True)
    assert ctx.factorize_now(_t(ref.vals), 1) == 1
    r = synth.random_vector(w.n_dofs, 6)
    z = ctx.precond_apply(_t(r)).cpu().numpy()
    ctx.close()
    print("[gpu-factor] hex_beam oracle banded solve", flush=True)
    p = ref.pat
    z_ref = solve.banded_cholesky_solve(p.n, p.row_ptr, p.col_idx, ref.vals, r)
    e = _rel(z, z_ref)
    print(f"  err vs banded solve {e:.2e}")
    assert e <= 1e-9


def test_gpu_factor_rejects_indefinite():
    w = synth.make("tiny_tet")
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=0, device=DEV, factor_on_gpu=True)
    A, _ = ctx.assemble(_params(w), _t(w.q0()), _t(w.v0()))
    with pytest.raises(_lib.FEError) as ei:
        ctx.factorize_now(-A, 1)
    assert ei.value.code == _lib.FE_EFACTOR
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_gpu_factor_trajectory(prec):
    """hex_diff, 5 steps, GPU refactorisation every 2 steps (lag 1)."""
    w = synth.make("hex_diff")
    qo, _ = step.rollout(w, w.q0(), w.v0(), 5, solver="banded")[-1]
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV, factor_on_gpu=True)
    p = _params(w)
    q, v = _t(w.q0()), _t(w.v0())
    its = []
    for _ in range(5):
        st = ctx.step(q, v, p, StepOptions(rel_tol=1e-8, max_it=500, refresh=2, lag=1))
        its.append(st.solve.iterations)
    torch.cuda.synchronize()
    e = np.linalg.norm(q.cpu().numpy() - qo) / np.linalg.norm(qo - w.q0())
    print(f"  prec={prec} iterations {its} displacement err {e:.2e}")
    assert e <= (1e-6 if prec == 0 else 1e-4)
    ctx.close()
