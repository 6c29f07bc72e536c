"""Full-size parity in the launch configuration bench.py times.

hex_beam (107,163 DOFs, mixed precision, graph-captured CG): assembled A and
b against the oracle's complete assembly; SpMV against the oracle's CSR
product; one step with a fresh factor against the oracle's banded-Cholesky
step; preconditioner residual; a short run of the benchmark schedule with a
residual certificate at every step.
tet_block (206,763 DOFs, jittered Kuhn tets, neo-Hookean), mixed and FP64:
assembly parity and the residual certificate of one step with a fresh
factor.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import assembly, solve, step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import FE_FACTOR_ASYNC, FE_FACTOR_DETERMINISTIC  # noqa: E402
from paper_2306_05893_amd.sim import Simulation  # noqa: E402

DEV = "cuda"


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def hex_beam():
    w = synth.make("hex_beam")
    print("[fullsize] hex_beam oracle pattern", flush=True)
    pat = step.pattern(w)
    return w, pat


def test_hex_beam_assembly_and_spmv(hex_beam):
    w, pat = hex_beam
    sim = Simulation(w, prec=1)
    ctx = sim.ctx
    q, v = synth.random_state(w, 0.002, 7)
    print("[fullsize] oracle assembly", flush=True)
    ref = step.assemble(w, q, v, pat=pat)
    A, b = ctx.assemble(sim.params, _t(q), _t(v))
    torch.cuda.synchronize()
    Ag = A.double().cpu().numpy()
    ea, eb = _rel(Ag, ref.vals), _rel(b.cpu().numpy(), ref.b)
    print(f"  A err {ea:.2e}  b err {eb:.2e}")
    assert ea <= 1e-5 and eb <= 1e-5
    x = synth.random_vector(w.n_dofs, 2)
    y = ctx.spmv(A, _t(x)).cpu().numpy()
    assert _rel(y, assembly.csr_matvec(pat.row_ptr, pat.col_idx, Ag, x)) <= 1e-12
    ctx.close()


def test_hex_beam_step_fresh_factor(hex_beam):
    """One step from a trajectory state, exact factor (refresh 1, lag 0):
    acceleration vs the oracle's banded Cholesky solve."""
    w, pat = hex_beam
    sim = Simulation(w, prec=1)
    q, v = synth.random_state(w, 0.002, 8)
    sim.q.copy_(_t(q))
    sim.v.copy_(_t(v))
    a = torch.zeros_like(sim.q)
    st = sim.step(sim.opts(rel_tol=1e-8, max_it=500, refresh=1, lag=0,
                           mode=FE_FACTOR_DETERMINISTIC), a_out=a)
    torch.cuda.synchronize()
    print("[fullsize] oracle banded step", flush=True)
    ref = step.assemble(w, q, v, pat=pat)
    a_ref = solve.banded_cholesky_solve(pat.n, pat.row_ptr, pat.col_idx, ref.vals, ref.b)
    ag = a.cpu().numpy()
    ea = _rel(ag, a_ref)
    res = np.linalg.norm(ref.b - assembly.csr_matvec(pat.row_ptr, pat.col_idx, ref.vals, ag)) / \
        np.linalg.norm(ref.b)
    print(f"  it={st.solve.iterations} gpu rel_res={st.solve.rel_res:.2e} "
          f"accel err vs oracle {ea:.2e}, residual vs exact A {res:.2e}")
    assert st.solve.rel_res <= 1e-8 and st.solve.iterations <= 3
    assert ea <= 1e-4
    sim.ctx.close()


def test_hex_beam_benchmark_schedule(hex_beam):
    """The benchmark's schedule (warmup deterministic, then asynchronous
    refresh): every step meets the recomputed-residual test and the
    trajectory stays within tolerance of the oracle's for 4 steps."""
    w, pat = hex_beam
    sim = Simulation(w, prec=1)
    det = sim.opts(rel_tol=1e-8, max_it=3000, refresh=10, lag=0, mode=FE_FACTOR_DETERMINISTIC)
    asy = sim.opts(rel_tol=1e-8, max_it=3000, refresh=10, lag=0, mode=FE_FACTOR_ASYNC)
    for k in range(4):
        st = sim.step(det if k < 2 else asy)
        assert st.solve.status == 0 and st.solve.rel_res <= 1e-8
    torch.cuda.synchronize()
    qg = sim.q.cpu().numpy()
    print("[fullsize] oracle 4-step rollout (banded)", flush=True)
    qo, _ = step.rollout(w, w.q0(), w.v0(), 4, solver="banded")[-1]
    e = np.linalg.norm(qg - qo) / np.linalg.norm(qo - w.q0())
    print(f"  4-step displacement rel err {e:.2e}")
    assert e <= 1e-4
    sim.ctx.close()


@pytest.fixture(scope="module")
def tet_block():
    w = synth.make("tet_block")
    print("[fullsize] tet_block oracle pattern and assembly at rest", flush=True)
    pat = step.pattern(w)
    ref = step.assemble(w, w.q0(), w.v0(), pat=pat)
    return w, pat, ref


@pytest.mark.parametrize("prec", [1, 0])
def test_tet_block_assembly_and_solve(tet_block, prec):
    """Assembly parity at rest, then one step from rest with a fresh factor
    (refresh 1, lag 0): the acceleration's residual is recomputed by the
    oracle's CSR product with the GPU's own A (FP32-valued in mixed
    precision) and with the oracle's exact A."""
    w, pat, ref = tet_block
    print(f"[fullsize] tet_block prec={prec}", flush=True)
    sim = Simulation(w, prec=prec, factor_on_gpu=True)
    ctx = sim.ctx
    A, b = ctx.assemble(sim.params, sim.q, sim.v)
    torch.cuda.synchronize()
    Ag = A.double().cpu().numpy()
    bg = b.cpu().numpy()
    ea, eb = _rel(Ag, ref.vals), _rel(bg, ref.b)
    print(f"  A err {ea:.2e} b err {eb:.2e}")
    tol = 1e-5 if prec == 1 else 1e-12
    assert ea <= tol and eb <= tol
    a = torch.zeros_like(sim.q)
    st = sim.step(sim.opts(rel_tol=1e-8, max_it=200, refresh=1, lag=0,
                           mode=FE_FACTOR_DETERMINISTIC), a_out=a)
    torch.cuda.synchronize()
    ah = a.cpu().numpy()
    res = np.linalg.norm(bg - assembly.csr_matvec(pat.row_ptr, pat.col_idx, Ag, ah)) / \
        np.linalg.norm(bg)
    res_exact = np.linalg.norm(ref.b - assembly.csr_matvec(pat.row_ptr, pat.col_idx, ref.vals,
                                                           ah)) / np.linalg.norm(ref.b)
    print(f"  it={st.solve.iterations} rel_res={st.solve.rel_res:.2e} oracle-recomputed "
          f"{res:.2e} (vs the oracle's A {res_exact:.2e})")
    assert st.solve.status == 0 and st.solve.iterations <= 3
    assert res <= 1e-8 * 1.01
    if prec == 0:
        assert res_exact <= 1e-8 * 1.01
    ctx.close()
