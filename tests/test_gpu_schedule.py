"""The stale-factor schedule of Sec. 3.3 (Eq. "asynchronous preconditioner")
on the GPU: which matrix a factor is taken from, and the asynchronous swap.

* Deterministic mode, refresh 3, lag 1: the factor in use after step 4 is
  that of A_3.  The snapshot of A_3 is taken on another stream while step 4
  assembles A_4 into the same buffer, so this pins the ordering of the
  snapshot copy against the next assembly.  Reference: the host LDL^T of
  A_3 (re-assembled from the saved state; the assembly sums in a fixed order,
  so it is the same matrix bit for bit) applied to the same vector.
* Asynchronous mode with the GPU factorisation (tet beam, refresh 3, 12
  steps): factors are swapped in while the rollout runs; every step meets the
  recomputed-residual test and the trajectory matches the oracle's
  direct-solve rollout (1e-7 in FP64, 1e-4 in mixed precision, whose FP32
  element arithmetic and A values move the trajectory itself).
* Asynchronous mode with the host factor thread on one core (differentiation
  beam, refresh 1, until two factors have been used): a refresh that falls
  due while the previous factorisation runs is skipped, so the second factor
  is that of the step at which the first job had finished; every step meets
  the recomputed-residual test and the trajectory matches a rollout with a
  fresh factor every step.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import step as ostep

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import (FE_FACTOR_ASYNC, FE_FACTOR_DETERMINISTIC,  # noqa: E402
                                  FE_PREC_FP64, FE_PREC_MIXED)
from paper_2306_05893_amd.sim import Simulation  # noqa: E402


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("gpu_factor", [True, False])
@pytest.mark.parametrize("prec", [FE_PREC_FP64, FE_PREC_MIXED])
def test_factor_is_of_the_snapshot_step(prec, gpu_factor):
    w = synth.make("hex_diff")
    print(f"[schedule] snapshot prec={prec} gpu_factor={gpu_factor}", flush=True)
    sim = Simulation(w, prec=prec, factor_on_gpu=gpu_factor)
    opts = sim.opts(rel_tol=1e-10, max_it=2000, refresh=3, lag=1, mode=FE_FACTOR_DETERMINISTIC)
    saved = None
    for k in range(5):
        if k == 3:
            saved = (sim.q.clone(), sim.v.clone())
        st = sim.step(opts)
        assert st.solve.status == 0
    assert st.solve.factor_tag == 3 and st.factor_lag == 1
    torch.cuda.synchronize()
    A3, _ = sim.ctx.assemble(sim.params, saved[0], saved[1])
    r = synth.random_vector(w.n_dofs, 12)
    z = sim.ctx.precond_apply(torch.as_tensor(r, device="cuda")).cpu().numpy()
    z_ref = sim.ctx.host_factor_apply(A3.double().cpu().numpy(), r[None])[0]
    e = _rel(z, z_ref)
    print(f"  installed factor (tag 3) vs host LDL^T of A_3: {e:.2e}")
    assert e <= (1e-10 if prec == FE_PREC_FP64 else 1e-5)
    sim.ctx.close()


def _check_rollout(w, sim, opts, nsteps, tol_traj):
    tags, lags = [], []
    for k in range(nsteps):
        st = sim.step(opts)
        assert st.solve.status == 0 and st.solve.rel_res <= opts.rel_tol, \
            f"step {k}: status {st.solve.status} rel_res {st.solve.rel_res:.2e}"
        tags.append(int(st.solve.factor_tag))
        lags.append(int(st.factor_lag))
    torch.cuda.synchronize()
    print(f"  factor tags used {tags}; lags {lags}", flush=True)
    used = [t for t in tags if t >= 0]
    # factors are taken at refresh steps, swapped in later, never swapped back
    assert all(t % opts.refresh == 0 for t in used)
    assert all(b >= a for a, b in zip(used, used[1:]))
    assert all(l >= 1 for t, l in zip(tags, lags) if t >= 0)
    qo, _ = ostep.rollout(w, w.q0(), w.v0(), nsteps, solver=ostep.default_solver(w.n_dofs))[-1]
    e = np.linalg.norm(sim.q.cpu().numpy() - qo) / np.linalg.norm(qo - w.q0())
    print(f"  {nsteps}-step displacement rel err vs oracle {e:.2e}")
    assert e <= tol_traj
    return used


@pytest.mark.parametrize("prec", [FE_PREC_FP64, FE_PREC_MIXED])
def test_async_swap_gpu_factor(prec):
    w = synth.make("tet_beam")
    print(f"[schedule] async GPU factor prec={prec}", flush=True)
    sim = Simulation(w, prec=prec, factor_on_gpu=True)
    opts = sim.opts(rel_tol=1e-10, max_it=3000, refresh=3, lag=0, mode=FE_FACTOR_ASYNC)
    # mixed precision: the FP32 element arithmetic and A values move the
    # trajectory itself (the bound of the other mixed trajectory tests)
    used = _check_rollout(w, sim, opts, 12, 1e-7 if prec == FE_PREC_FP64 else 1e-4)
    assert len(set(used)) >= 3, "expected at least three factors swapped in"
    sim.ctx.close()


def test_async_skips_refresh_while_busy():
    # Refresh every step, one host factor thread: a factorisation of the
    # 14,883-DOF beam takes many steps, so the refreshes that fall due while
    # it runs are skipped (not queued): the next factor used is that of the
    # step at which the previous job had finished, not of the next step.
    # Runs until two factors have been used.  Reference: the same steps with
    # a fresh GPU factor every step (deterministic schedule); both solve every
    # step to the same recomputed-residual test.
    w = synth.make("hex_diff")
    print("[schedule] async host factor (one thread), refresh 1", flush=True)
    sim = Simulation(w, prec=FE_PREC_FP64, factor_on_gpu=False, n_threads=1)
    opts = sim.opts(rel_tol=1e-10, max_it=5000, refresh=1, lag=0, mode=FE_FACTOR_ASYNC)
    tags = []
    while len({t for t in tags if t >= 0}) < 2 and len(tags) < 1500:
        st = sim.step(opts)
        assert st.solve.status == 0 and st.solve.rel_res <= opts.rel_tol
        tags.append(int(st.solve.factor_tag))
    torch.cuda.synchronize()
    used = sorted({t for t in tags if t >= 0})
    first_use = [tags.index(t) for t in used]
    print(f"  {len(tags)} steps, factors {used} first used at steps {first_use}")
    assert len(used) == 2, "expected a second factor within 1500 steps"
    assert used[0] == 0 and first_use[0] >= 2, "the first factor should take several steps"
    # the second job started at the first step after the first had finished
    # (every refresh due in between was skipped)
    assert used[1] >= first_use[0] - 1 and used[1] - used[0] >= 2
    ref = Simulation(w, prec=FE_PREC_FP64, factor_on_gpu=True)
    ropts = ref.opts(rel_tol=1e-10, max_it=500, refresh=1, lag=0, mode=FE_FACTOR_DETERMINISTIC)
    for _ in range(len(tags)):
        ref.step(ropts)
    torch.cuda.synchronize()
    u = (ref.q - ref.q.new_tensor(w.q0())).norm()
    e = float((sim.q - ref.q).norm() / u)
    print(f"  displacement vs fresh-factor rollout {e:.2e}")
    assert e <= 1e-6
    sim.ctx.close()
    ref.ctx.close()
