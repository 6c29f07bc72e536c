"""Full assembly on a topology change (paper Sec. 4: the keepStruct test of
Alg. "add" and the rebuild of the pattern and map when the fill order
changes, e.g. cutting).

* keepStruct on the GPU: the same connectivity keeps the map; a removed
  element, a permuted node order (same pattern, another fill sequence) or
  other fixed DOFs are detected.
* Cutting mid-trajectory: the hex beam of the differentiation workload runs 3
  steps, a slab of elements across the beam is removed (the tip floats
  free), and 3 more steps run on the rebuilt context; both segments are
  compared with the oracle doing the same."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from oracle import step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import FE_PREC_FP64, FE_PREC_MIXED  # noqa: E402
from paper_2306_05893_amd.sim import Simulation  # noqa: E402

DEV = "cuda"


def _cut(w, k_lo, k_hi):
    """Elements whose centroid z lies in [k_lo, k_hi) cells are removed."""
    zc = w.X[w.conn][:, :, 2].mean(axis=1) / w.spacing
    keep = ~((zc >= k_lo) & (zc < k_hi))
    return np.ascontiguousarray(w.conn[keep]), np.ascontiguousarray(w.E[keep]), keep


def test_keepstruct_detection():
    w = synth.make("hex_diff")
    sim = Simulation(w, prec=FE_PREC_MIXED, factor_on_gpu=True)
    ctx = sim.ctx

    def dconn(c):
        return torch.as_tensor(np.ascontiguousarray(c, dtype=np.int32).reshape(-1), device=DEV)

    assert not ctx.structure_changed(dconn(w.conn))
    c2 = w.conn.copy()
    c2[100, [1, 3]] = c2[100, [3, 1]]           # same nodes, another fill order
    assert ctx.structure_changed(dconn(c2))
    assert ctx.structure_changed(dconn(w.conn[:-1]))
    fx = torch.as_tensor(w.fixed, device=DEV)
    assert not ctx.structure_changed(dconn(w.conn), fx)
    fx2 = w.fixed.copy()
    fx2[np.flatnonzero(fx2 == 0)[7]] = 1
    assert ctx.structure_changed(dconn(w.conn), torch.as_tensor(fx2, device=DEV))
    # set_topology keeps the context when nothing changed
    old = sim.ctx
    assert sim.set_topology(w.conn, w.E) is False and sim.ctx is old
    sim.ctx.close()


@pytest.mark.parametrize("prec", [FE_PREC_FP64, FE_PREC_MIXED])
def test_cut_mid_trajectory(prec):
    w = synth.make("hex_diff")
    conn2, E2, keep = _cut(w, 20, 21)
    print(f"[topology] cut removes {int((~keep).sum())} of {w.n_elems} elements", flush=True)
    sim = Simulation(w, prec=prec, factor_on_gpu=True)
    opts = sim.opts(rel_tol=1e-12 if prec == FE_PREC_FP64 else 1e-9, max_it=3000, refresh=1,
                    lag=0)
    for _ in range(3):
        st = sim.step(opts)
        assert st.solve.status == 0
    nnz0 = sim.ctx.sizes.nnz
    assert sim.set_topology(conn2, E2) is True
    print(f"[topology] rebuilt: nnz {nnz0} -> {sim.ctx.sizes.nnz}", flush=True)
    assert sim.ctx.sizes.nnz < nnz0
    for _ in range(3):
        st = sim.step(sim.opts(rel_tol=opts.rel_tol, max_it=3000, refresh=1, lag=0))
        assert st.solve.status == 0
    torch.cuda.synchronize()
    q = sim.q.cpu().numpy()
    # oracle: 3 steps on the full mesh, 3 on the cut mesh
    q3, v3 = step.rollout(w, w.q0(), w.v0(), 3, solver="banded")[-1]
    w2 = dataclasses.replace(w, conn=conn2, E=E2)
    qo, _ = step.rollout(w2, q3, v3, 3, solver="banded")[-1]
    e = np.linalg.norm(q - qo) / np.linalg.norm(qo - w.q0())
    # the tip has been released: it moves differently from the uncut beam
    qu, _ = step.rollout(w, q3, v3, 3, solver="banded")[-1]
    sep = np.linalg.norm(qu - qo) / np.linalg.norm(qo - w.q0())
    print(f"  prec {prec}: displacement err {e:.2e} (cut vs uncut differ by {sep:.2e})")
    assert e <= (1e-8 if prec == FE_PREC_FP64 else 1e-4)
    assert sep > 100 * e
    sim.ctx.close()
