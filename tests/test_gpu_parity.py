"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (normwise max-relative ||gpu - oracle||_max / ||oracle||_max):
  FP64 path 1e-12 for A, b and SpMV; FP32 (mixed) path 1e-5.
Solves are certified by the oracle recomputing ||b - A x|| / ||b|| with the
GPU's own A upcast to FP64 (<= the requested tolerance); the residual against
the oracle's exact A is printed as well.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import assembly, solve, step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import _lib  # noqa: E402
from paper_2306_05893_amd.sim import FEContext, Params, StepOptions, rollout  # noqa: E402

DEV = "cuda"


def _ctx(w, prec):
    print(f"[ctx] {w.name} elem={w.elem_type} mat={w.material} prec={prec}", flush=True)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV)
    ctx.bind()
    return ctx


def _params(w, E=None):
    return Params(w.h, w.alpha, w.beta, w.rho, w.nu, w.material, w.gravity,
                  w.E if E is None else E, w.f_nodal, DEV)


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _state(w, seed=1, steps=2):
    q, v = step.rollout(w, w.q0(), w.v0(), steps)[-1]
    return q, v


CASES = [("tiny_tet", 0), ("tiny_tet", 1), ("tiny_hex", 0), ("tiny_hex", 1), ("tet_beam", 0),
         ("tet_beam", 1), ("hex_diff", 0), ("hex_diff", 1)]


@pytest.mark.parametrize("mesh,mat", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_assembly_parity(mesh, mat, prec):
    w = synth.make(mesh, material=mat)
    q, v = _state(w)
    v = v + 0.05 * synth.random_vector(w.n_dofs, 5) * (1 - w.fixed)
    ref = step.assemble(w, q, v)
    ctx = _ctx(w, prec)
    A, b = ctx.assemble(_params(w), _t(q), _t(v))
    torch.cuda.synchronize()
    A = A.double().cpu().numpy()
    b = b.cpu().numpy()
    ea, eb = _rel(A, ref.vals), _rel(b, ref.b)
    print(f"  A err {ea:.3e}  b err {eb:.3e}")
    tol = 1e-12 if prec == 0 else 1e-5
    assert ea <= tol and eb <= tol


@pytest.mark.parametrize("prec", [0, 1])
def test_assembly_parity_per_dof_constraints(prec):
    """Roller constraints: the int32 map path of the element kernel."""
    w = synth.make("tiny_hex", material=1)
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


@pytest.mark.parametrize("mesh", ["tet_beam", "hex_diff"])
@pytest.mark.parametrize("prec", [0, 1])
def test_spmv_parity(mesh, prec):
    w = synth.make(mesh)
    q, v = _state(w)
    ref = step.assemble(w, q, v)
    ctx = _ctx(w, prec)
    vals = ref.vals.astype(np.float32 if prec else np.float64)
    A = torch.as_tensor(vals, device=DEV)
    x = synth.random_vector(w.n_dofs, 3)
    y = ctx.spmv(A, _t(x)).cpu().numpy()
    y_ref = assembly.csr_matvec(ref.pat.row_ptr, ref.pat.col_idx, vals.astype(np.float64), x)
    e = _rel(y, y_ref)
    print(f"  spmv err vs same-valued A {e:.3e}; vs FP64 A "
          f"{_rel(y, assembly.csr_matvec(ref.pat.row_ptr, ref.pat.col_idx, ref.vals, x)):.3e}")
    assert e <= 1e-12


@pytest.mark.parametrize("mesh", ["tiny_tet", "tet_beam", "hex_diff"])
@pytest.mark.parametrize("prec", [0, 1])
def test_preconditioner_parity(mesh, prec):
    """z = P^{-1} r on the GPU vs the oracle's dense/banded solve with A_t0."""
    w = synth.make(mesh)
    q, v = _state(w)
    ref = step.assemble(w, q, v)
    ctx = _ctx(w, prec)
    A, _ = ctx.assemble(_params(w), _t(q), _t(v))
    tag = ctx.factorize_now(A, 7)
    assert tag == 7
    r = synth.random_vector(w.n_dofs, 4)
    z = ctx.precond_apply(_t(r)).cpu().numpy()
    p = ref.pat
    Ag = A.double().cpu().numpy()
    z_ref = (solve.dense_cholesky_solve if w.n_dofs < 4000 else solve.banded_cholesky_solve)(
        p.n, p.row_ptr, p.col_idx, Ag, r)
    e = _rel(z, z_ref)
    z_host = ctx.host_factor_apply(Ag, r[None])[0]
    print(f"  precond err vs dense {e:.3e}; vs host panels {_rel(z, z_host):.3e}")
    assert e <= (1e-9 if prec == 0 else 1e-5)
    assert _rel(z, z_host) <= (1e-11 if prec == 0 else 1e-5)


@pytest.mark.parametrize("extents", [(16, 256, 16, 1), (32, 1024, 32, 1), (128, 512, 16, 1),
                                     (64, 256, 32, 2), (0, 0, 0, 0), (0, 0, 32, 4),
                                     (64, 1024, 64, 4)])
@pytest.mark.parametrize("prec", [0, 1])
def test_preconditioner_parity_tile_extents(extents, prec):
    """Every sweep tile shape (and the per-level choice, extents 0) gives the
    same z = P^{-1} r as the oracle's banded solve with A_t0."""
    w = synth.make("hex_diff")
    q, v = _state(w)
    ref = step.assemble(w, q, v)
    fc, br, bc, fg = extents
    print(f"[ctx] {w.name} prec={prec} fwd_tile_cols={fc} fwd_col_groups={fg} "
          f"bwd_tile_rows={br} bwd_tile_cols={bc}", flush=True)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV,
                    fwd_tile_cols=fc, bwd_tile_rows=br, bwd_tile_cols=bc, fwd_col_groups=fg)
    ctx.bind()
    A, _ = ctx.assemble(_params(w), _t(q), _t(v))
    ctx.factorize_now(A, 0)
    r = synth.random_vector(w.n_dofs, 4)
    z = ctx.precond_apply(_t(r)).cpu().numpy()
    p = ref.pat
    z_ref = solve.banded_cholesky_solve(p.n, p.row_ptr, p.col_idx, A.double().cpu().numpy(), r)
    e = _rel(z, z_ref)
    print(f"  precond err vs banded {e:.3e}")
    assert e <= (1e-9 if prec == 0 else 1e-5)


@pytest.mark.parametrize("mesh", ["tet_beam", "hex_diff"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("use_factor", [True, False])
def test_pcg_residual_certificate(mesh, prec, use_factor):
    w = synth.make(mesh)
    q, v = _state(w)
    ref = step.assemble(w, q, v)
    ctx = _ctx(w, prec)
    A, b = ctx.assemble(_params(w), _t(q), _t(v))
    if use_factor:
        ctx.factorize_now(A, 0)
    x, st = ctx.pcg_solve(A, b, rel_tol=1e-8, max_it=20000)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    Ag = A.double().cpu().numpy()
    bg = b.cpu().numpy()
    p = ref.pat
    res_own = np.linalg.norm(bg - assembly.csr_matvec(p.row_ptr, p.col_idx, Ag, xg)) / np.linalg.norm(bg)
    res_ora = np.linalg.norm(ref.b - assembly.csr_matvec(p.row_ptr, p.col_idx, ref.vals, xg)) / \
        np.linalg.norm(ref.b)
    print(f"  it={st.iterations} gpu rel_res={st.rel_res:.2e} oracle(own A)={res_own:.2e} "
          f"oracle(exact A)={res_ora:.2e}")
    assert st.status == 0
    assert res_own <= 1e-8 * 1.01
    assert abs(st.rel_res - res_own) <= 1e-9
    if use_factor and prec == 0:
        assert st.iterations <= 2          # exact preconditioner


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("use_factor", [True, False])
def test_graph_replays_match_eager(prec, use_factor):
    """CG iterations replayed from a captured HIP graph give the eager result
    on every replay (stale factor: several iterations per solve), with eager
    library work and host synchronisation between the replays."""
    w = synth.make("hex_diff")
    ctx = _ctx(w, prec)
    p = _params(w)
    if use_factor:
        A0, _ = ctx.assemble(p, _t(w.q0()), _t(w.v0()))
        ctx.factorize_now(A0, 0)
    q, v = _state(w, steps=4)
    A, b = ctx.assemble(p, _t(q), _t(v))
    runs = []
    for mode in ["eager", "graph", "graph", "eager", "graph", "graph"]:
        ctx.set_graphs(mode == "graph")
        x, st = ctx.pcg_solve(A, b, rel_tol=1e-10, max_it=3000)
        torch.cuda.synchronize()
        runs.append((mode, x.cpu().numpy(), st.iterations, st.rel_res))
        ctx.spmv(A, x)                         # eager work between replays
        torch.cuda.synchronize()
    ref = runs[0]
    print("  " + ", ".join(f"{m}:{it}" for m, _, it, _ in runs))
    assert ref[2] > 2
    for mode, x, it, rr in runs[1:]:
        assert abs(it - ref[2]) <= 2, (mode, it, ref[2])
        assert rr <= 1e-10 * 1.01
        assert _rel(x, ref[1]) <= 1e-7


def test_zero_rhs_gives_zero_solution():
    w = synth.make("tiny_hex")
    ctx = _ctx(w, 0)
    A, _ = ctx.assemble(_params(w), _t(w.q0()), _t(w.v0()))
    b = torch.zeros(w.n_dofs, dtype=torch.float64, device=DEV)
    x, st = ctx.pcg_solve(A, b)
    assert st.iterations == 0 and float(x.abs().max()) == 0.0


def _gpu_rollout(w, prec, nsteps, opts):
    ctx = _ctx(w, prec)
    p = _params(w)
    q, v = _t(w.q0()), _t(w.v0())
    stats = []
    for _ in range(nsteps):
        st = ctx.step(q, v, p, opts)
        stats.append((st.solve.iterations, st.solve.rel_res, st.factor_lag))
    torch.cuda.synchronize()
    return q.cpu().numpy(), v.cpu().numpy(), stats


def test_tet_beam_trajectory_fp64_exact_factor():
    """Tet beam, plain FP64: 10 steps, exact LDL^T (R=1, d=0), rel-res 1e-10."""
    w = synth.make("tet_beam")
    qo, vo = step.rollout(w, w.q0(), w.v0(), w.steps)[-1]
    q, v, stats = _gpu_rollout(w, 0, w.steps, StepOptions(rel_tol=1e-10, max_it=100, refresh=1,
                                                          lag=0))
    u_ref = qo - w.q0()
    eq = np.linalg.norm(q - qo) / np.linalg.norm(u_ref)
    ev = np.linalg.norm(v - vo) / np.linalg.norm(vo)
    print(f"  displacement rel err {eq:.3e}, velocity rel err {ev:.3e}, stats {stats}")
    assert all(s[0] <= 2 for s in stats)
    assert eq <= 1e-7 and ev <= 1e-7


@pytest.mark.parametrize("prec", [0, 1])
def test_hex_diff_trajectory_stale_factor(prec):
    """Hex beam 4000 HEX8, 5 steps, factor refreshed every 3 steps (stale in
    between), rel-res 1e-8 (FP64) / 1e-8 (mixed)."""
    w = synth.make("hex_diff")
    n = 5
    qo, vo = step.rollout(w, w.q0(), w.v0(), n, solver="banded")[-1]
    q, v, stats = _gpu_rollout(w, prec, n, StepOptions(rel_tol=1e-8, max_it=500, refresh=3, lag=1))
    eq = np.linalg.norm(q - qo) / np.linalg.norm(qo - w.q0())
    print(f"  prec={prec} displacement rel err {eq:.3e}; stats {stats}")
    assert eq <= (1e-6 if prec == 0 else 1e-4)


def test_inverted_element_is_reported():
    w = synth.make("tiny_hex")
    ctx = _ctx(w, 0)
    q = w.q0().copy()
    free_nodes = np.flatnonzero(w.fixed.reshape(-1, 3)[:, 0] == 0)
    q[3 * free_nodes[0] + 2] -= 5 * w.spacing      # push one node through its element
    with pytest.raises(_lib.FEError) as ei:
        ctx.assemble(_params(w), _t(q), _t(w.v0()))
    assert ei.value.code == _lib.FE_EINVERTED


def test_adjoint_matches_oracle_and_complex_step():
    """dL/dE, dL/dq0, dL/dv0 of L = ||q_T - q_target||^2 over 4 steps with
    checkpoints every 2 steps, vs the oracle adjoint and a complex-step
    derivative of the oracle rollout."""
    w = synth.make("tiny_hex")
    nsteps, k = 4, 2
    E = synth.lognormal_E(w.n_elems, 5000.0, 0.3, 0)
    q0, v0 = w.q0(), w.v0()
    st_ora = step.rollout(w, q0, v0, nsteps, E)
    target = st_ora[-1][0] + 1e-4 * synth.random_vector(w.n_dofs, 3)
    dE_o, dq_o, dv_o = oadj.adjoint_rollout(w, E, st_ora, 2 * (st_ora[-1][0] - target),
                                            np.zeros(w.n_dofs))
    ctx = _ctx(w, 0)
    p = _params(w, E)
    Et = _t(E).requires_grad_(True)
    q0t = _t(q0).requires_grad_(True)
    v0t = _t(v0).requires_grad_(True)
    opts = StepOptions(rel_tol=1e-12, max_it=200, refresh=1, lag=0)
    qT, vT = rollout(Et, q0t, v0t, ctx, p, nsteps, k, opts)
    loss = ((qT - _t(target)) ** 2).sum()
    loss.backward()
    dE = Et.grad.cpu().numpy()
    dq = q0t.grad.cpu().numpy()
    dv = v0t.grad.cpu().numpy()
    print(f"  dE err {_rel(dE, dE_o):.2e} dq0 err {_rel(dq, dq_o):.2e} dv0 err {_rel(dv, dv_o):.2e}")
    assert _rel(dE, dE_o) <= 1e-6 and _rel(dq, dq_o) <= 1e-6 and _rel(dv, dv_o) <= 1e-6
    e = np.zeros(w.n_elems)
    e[2] = 1.0
    cs = oadj.rollout_loss_complex_step(w, E, q0, v0, target, nsteps, dE=e)
    assert abs(dE[2] - cs) <= 1e-5 * abs(cs)
