"""The compliance entry point that allocates nothing (fe_compliance_noalloc)
against fe_compliance, which takes a caller workspace: same W = H P^{-1} H^T
and Z = P^{-1} H^T on the 14,883-DOF differentiation beam, two calls in a
row (the second with fewer constraint rows, so it reuses a smaller part of
the static scratch that the first call left filled), both precisions, GPU
factor.  Tolerances relative to the largest entry: FP64 1e-12, mixed 1e-5
(the sweeps add into their outputs with atomics, so two runs of the same
kernels differ by FP32 rounding).  The first call is also checked against
the contact oracle.  A k whose blocks exceed the scratch is refused before
any launch."""
import numpy as np
import pytest
import torch

import synth
from oracle import contact, step

pytestmark = pytest.mark.gpu

from paper_2306_05893_amd import FEError  # noqa: E402
from paper_2306_05893_amd.sim import Constraints, FEContext  # noqa: E402

DEV = "cuda"


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("prec", [0, 1])
def test_compliance_noalloc_matches_workspace_entry_point(prec):
    w = synth.make("hex_diff")
    q, v = synth.random_state(w, 0.002, 4)
    ref = step.assemble(w, q, v)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, device=DEV,
                    factor_on_gpu=True)
    vals = ref.vals.astype(np.float32) if prec else ref.vals
    ctx.factorize_now(torch.as_tensor(vals, device=DEV), 1)
    tol = 1e-12 if prec == 0 else 1e-5
    for call, (k, seed) in enumerate(((200, 21), (37, 22))):
        print(f"[no-alloc] hex_diff prec={prec} call {call}: k={k}", flush=True)
        Hh, _ = synth.contact_constraints(w, k, seed, "mixed")
        H = Constraints.from_host(Hh, DEV)
        W_ref, Z_ref = ctx.compliance(H, want_Z=True)
        W = torch.full((k, k), np.nan, dtype=torch.float64, device=DEV)
        Z = torch.full((w.n_dofs, k), np.nan, dtype=torch.float64, device=DEV)
        ctx.compliance_noalloc(H, W, Z)
        Wg, Zg = W.cpu().numpy(), Z.cpu().numpy()
        ew, ez = _rel(Wg, W_ref.cpu().numpy()), _rel(Zg, Z_ref.cpu().numpy())
        print(f"  vs fe_compliance: W {ew:.2e}  Z {ez:.2e}", flush=True)
        assert np.isfinite(Wg).all() and np.isfinite(Zg).all()
        assert ew <= tol and ez <= tol
        if call == 0:
            p = ref.pat
            Wo, _ = contact.compliance(p.n, p.row_ptr, p.col_idx, vals.astype(np.float64), Hh,
                                       "banded")
            eo = _rel(Wg, Wo)
            print(f"  W vs oracle {eo:.2e}", flush=True)
            assert eo <= (1e-9 if prec == 0 else 1e-5)
    # more right-hand sides than the static scratch holds: refused on the host
    k_big = 1200
    Hbig = Constraints.from_host((np.zeros(k_big + 1, np.int32), np.zeros(0, np.int32),
                                  np.zeros(0)), DEV)
    Wbig = torch.zeros(k_big, k_big, dtype=torch.float64, device=DEV)
    with pytest.raises(FEError, match="static scratch"):
        ctx.compliance_noalloc(Hbig, Wbig)
    # the context still works afterwards
    Hh, _ = synth.contact_constraints(w, 5, 23, "plane")
    H = Constraints.from_host(Hh, DEV)
    W = torch.zeros(5, 5, dtype=torch.float64, device=DEV)
    ctx.compliance_noalloc(H, W)
    assert _rel(W.cpu().numpy(), ctx.compliance(H).cpu().numpy()) <= tol
    ctx.close()
