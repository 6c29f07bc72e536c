"""Differentiation workload at full size: 10x10x40 hex beam (4000 HEX8,
14,883 DOFs), per-element E log-normal (median 5000 Pa, sigma_ln 0.3),
20 implicit steps, checkpoints every 5 steps, FP64, solves to rel-res 1e-12.
Loss L = ||q_T - q_target||^2 with q_target from a second E field.

dL/dE from the adjoint rollout (autograd Function over fe_step_adjoint) is
checked against
* central finite differences of the GPU forward rollout on 20 random
  elements (dE = 1e-4 E_e), to 1e-4 relative (the denominator floored at
  1% of the largest of the 20 differences, for components near zero whose
  difference quotient is dominated by rounding);
* the oracle's adjoint recursion (banded Cholesky solves), element by
  element on all 4000 elements.
"""
import time

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import FE_PREC_FP64  # noqa: E402
from paper_2306_05893_amd.sim import StepOptions, Simulation, rollout  # noqa: E402

DEV = "cuda"
NSTEPS, CKPT = 20, 5


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.fixture(scope="module")
def diff():
    w = synth.make("hex_diff")
    sim = Simulation(w, prec=FE_PREC_FP64, factor_on_gpu=True)
    opts = StepOptions(rel_tol=1e-12, max_it=500, refresh=1, lag=0)

    def forward(E):
        with torch.no_grad():
            qT, _ = rollout(_t(E), _t(w.q0()), _t(w.v0()), sim.ctx, sim.params, NSTEPS, CKPT,
                            opts)
        return qT

    t0 = time.time()
    q_target = forward(w.extra["E_target"])
    print(f"[diff] target rollout ({time.time() - t0:.1f}s)", flush=True)
    yield w, sim, opts, forward, q_target
    sim.ctx.close()


def test_adjoint_vs_finite_differences(diff):
    w, sim, opts, forward, q_target = diff
    E = w.E.copy()
    Et = _t(E).requires_grad_(True)
    qT, _ = rollout(Et, _t(w.q0()), _t(w.v0()), sim.ctx, sim.params, NSTEPS, CKPT, opts)
    loss = ((qT - q_target) ** 2).sum()
    loss.backward()
    g = Et.grad.cpu().numpy()
    print(f"[diff] adjoint gradient, loss {float(loss.detach()):.6e}", flush=True)
    fds = []
    for e in w.extra["fd_elements"]:
        d = 1e-4 * E[e]
        Ep, Em = E.copy(), E.copy()
        Ep[e] += d
        Em[e] -= d
        lp = float(((forward(Ep) - q_target) ** 2).sum())
        lm = float(((forward(Em) - q_target) ** 2).sum())
        fd = (lp - lm) / (2 * d)
        fds.append(fd)
        print(f"  element {e}: adjoint {g[e]:.6e} fd {fd:.6e}", flush=True)
    fds = np.array(fds)
    ga = g[w.extra["fd_elements"]]
    floor = 1e-2 * np.abs(fds).max()
    errs = np.abs(ga - fds) / np.maximum(np.abs(fds), floor)
    print(f"  max rel err {errs.max():.2e} (plain relative {np.max(np.abs(ga - fds) / np.abs(fds)):.2e})")
    assert errs.max() <= 1e-4


def test_adjoint_vs_oracle(diff):
    w, sim, opts, forward, _ = diff
    # the target of this comparison comes from the oracle (its inputs never
    # come from the GPU path); both sides use it
    t0 = time.time()
    qt = step.rollout(w, w.q0(), w.v0(), NSTEPS, w.extra["E_target"], solver="banded")[-1][0]
    st = step.rollout(w, w.q0(), w.v0(), NSTEPS, w.E, solver="banded")
    print(f"[diff] oracle rollouts ({time.time() - t0:.1f}s)", flush=True)
    t0 = time.time()
    g_o, _, _ = oadj.adjoint_rollout(w, w.E, st, 2 * (st[-1][0] - qt), np.zeros(w.n_dofs),
                                     solver="banded")
    print(f"[diff] oracle adjoint ({time.time() - t0:.1f}s)", flush=True)
    Et = _t(w.E).requires_grad_(True)
    qT, _ = rollout(Et, _t(w.q0()), _t(w.v0()), sim.ctx, sim.params, NSTEPS, CKPT, opts)
    loss = ((qT - _t(qt)) ** 2).sum()
    loss.backward()
    g = Et.grad.cpu().numpy()
    e_fwd = np.linalg.norm(st[-1][0] - qT.detach().cpu().numpy()) / \
        np.linalg.norm(st[-1][0] - w.q0())
    e = float(np.abs(g - g_o).max() / np.abs(g_o).max())
    print(f"  forward displacement rel err {e_fwd:.2e}; dL/dE rel err {e:.2e}")
    assert e_fwd <= 1e-9 and e <= 1e-6
