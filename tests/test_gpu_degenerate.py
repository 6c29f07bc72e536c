"""Degenerate meshes through the whole step, against the oracle (dense
solves): a single hex with one face fixed, a single tet with three nodes
fixed (one free node), a hex with every DOF fixed (A = I, b = 0, nothing
moves, no CG iteration) and a free-floating block with no Dirichlet DOF at
all (A is positive definite through the mass term alone).  Each runs two
steps in FP64 and in mixed precision, with a fresh factor every step, on
the host-thread factorisation and on the GPU one.  The CG's error paths
(an indefinite matrix, an iteration cap) on the tet beam."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from oracle import assembly, step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd.sim import FEContext, Params, StepOptions  # noqa: E402

DEV = "cuda"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _workload(kind):
    base = synth.make("tiny_hex")
    if kind in ("single_hex", "all_fixed"):
        X, conn = synth.hex_beam(1, 1, 1, spacing=0.01)
        fixed = synth.fixed_face_dofs(X, 2, 0.0)
        if kind == "all_fixed":
            fixed = np.ones_like(fixed)
        et = synth.HEX8
    elif kind == "single_tet":
        X0, conn0 = synth.tet_block(1, 1, 1, spacing=0.01)
        X = X0[conn0[0]]
        conn = np.arange(4, dtype=np.int32)[None, :]
        fixed = synth.fixed_face_dofs(X, 2, 0.0)
        et = synth.TET4
    else:  # free-floating block, no Dirichlet DOF
        X, conn = synth.hex_beam(2, 2, 2, spacing=0.01)
        fixed = np.zeros(3 * X.shape[0], np.uint8)
        et = synth.HEX8
    n_el = conn.shape[0]
    return dataclasses.replace(base, name=kind, elem_type=et, X=X, conn=conn.astype(np.int32),
                               fixed=fixed.astype(np.uint8), E=np.full(n_el, 5000.0),
                               f_nodal=np.zeros_like(X))


@pytest.mark.parametrize("kind", ["single_hex", "single_tet", "all_fixed", "free_floating"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gpu_factor", [False, True])
def test_degenerate_mesh_steps(kind, prec, gpu_factor):
    w = _workload(kind)
    print(f"[degenerate] {kind} prec={prec} gpu_factor={gpu_factor} n={w.n_dofs}", flush=True)
    states = step.rollout(w, w.q0(), w.v0(), 2, solver="dense")
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV,
                    factor_on_gpu=gpu_factor)
    p = Params(w.h, w.alpha, w.beta, w.rho, w.nu, w.material, w.gravity, w.E, w.f_nodal, DEV)
    q, v = _t(w.q0()), _t(w.v0())
    opts = StepOptions(rel_tol=1e-12 if prec == 0 else 1e-8, max_it=200, refresh=1, lag=0)
    its = []
    for k in range(2):
        st = ctx.step(q, v, p, opts)
        its.append(st.solve.iterations)
        qo, vo = states[k + 1]
        uq = np.abs(qo - w.q0()).max()
        eq = np.abs(q.cpu().numpy() - qo).max() / max(uq, 1e-300)
        ev = np.abs(v.cpu().numpy() - vo).max() / max(np.abs(vo).max(), 1e-300)
        print(f"  step {k}: its {st.solve.iterations} q err {eq:.2e} v err {ev:.2e}", flush=True)
        if kind == "all_fixed":
            assert float((q - _t(w.q0())).abs().max()) == 0.0
            assert float(v.abs().max()) == 0.0
            assert st.solve.iterations == 0
        else:
            # mixed: the step solves the FP32-rounded A exactly (rel-res 1e-8),
            # so the trajectory differs from the FP64 oracle by about cond(A)
            # times the FP32 rounding; the same bound as the other mixed
            # trajectory tests
            tol = 1e-9 if prec == 0 else 1e-4
            assert eq <= tol and ev <= tol
    ctx.close()


def _tet_beam_system(prec):
    w = synth.make("tet_beam")
    ref = step.assemble(w, w.q0(), w.v0())
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV)
    A = torch.as_tensor(ref.vals, dtype=ctx.value_dtype, device=DEV)
    return ref, ctx, A


@pytest.mark.parametrize("prec", [0, 1])
def test_cg_reports_indefinite(prec):
    """-A (negative definite, Jacobi preconditioner): the first p^T A p is
    negative, and the solve stops with FE_EINDEF."""
    from paper_2306_05893_amd import _lib
    print(f"[cg-errors] indefinite prec={prec}", flush=True)
    ref, ctx, A = _tet_beam_system(prec)
    with pytest.raises(_lib.FEError) as ei:
        ctx.pcg_solve(-A, _t(ref.b), rel_tol=1e-10, max_it=50)
    assert ei.value.code == _lib.FE_EINDEF
    ctx.close()


@pytest.mark.parametrize("prec,max_it", [(0, 4), (1, 4), (0, 5), (1, 7)])
def test_cg_reports_not_converged(prec, max_it):
    """An iteration cap far below what the tolerance needs: FE_ENOTCONV after
    exactly max_it iterations (odd caps too: the graph-captured batches of
    two iterations must not overshoot), the iterate and the recomputed
    residual still returned."""
    from paper_2306_05893_amd import _lib
    print(f"[cg-errors] not converged prec={prec} max_it={max_it}", flush=True)
    ref, ctx, A = _tet_beam_system(prec)
    x, st = ctx.pcg_solve(A, _t(ref.b), rel_tol=1e-14, max_it=max_it)
    assert st.status == _lib.FE_ENOTCONV
    assert st.iterations == max_it
    xh = x.cpu().numpy()
    assert np.isfinite(xh).all()
    # the reported residual is the recomputed one: FP64 arithmetic on the
    # context's values (FP32-rounded in mixed precision)
    vals = ref.vals if prec == 0 else ref.vals.astype(np.float32).astype(np.float64)
    p = ref.pat
    res = np.linalg.norm(ref.b - assembly.csr_matvec(p.row_ptr, p.col_idx, vals, xh))
    res /= np.linalg.norm(ref.b)
    print(f"  iterations {st.iterations}, rel-res {st.rel_res:.3e} (oracle {res:.3e})")
    assert res > 1e-14 and abs(st.rel_res - res) <= 1e-8 * res
    ctx.close()
