"""Throughput of the implicit FE step on one MI355X.

Headline workload: the large two-material hex block, 48 x 48 x 192 trilinear
hexahedra (2x2x2 Gauss points; 442,368 elements, 463,393 nodes, 1,390,179
DOFs), neo-Hookean with E = 2000 Pa and 20000 Pa in 64 seeded spherical
inclusions of radius 4 cells, nu = 0.45, gravity, z = 0 face fixed,
h = 0.01 s, Rayleigh alpha = beta = 0.1, mixed precision (FP32 element
kernels, A values and triangular solves; FP64 state, CG vectors, dots and
residual), CG to relative residual 1e-8, LDL^T preconditioner refactored
every 20 steps and swapped in when ready (the paper's asynchronous scheme;
the FP64 multifrontal factorisation runs on its own GPU stream in place of
the paper's CPU thread).  Each step's CG starts from the A-norm projection
of its solution onto the last 8 accelerations (the paper leaves the initial
guess open; every step still meets the same recomputed-residual test).
Beside it, on the same workload: the same steps from x0 = 0, FP64 steps/s,
and the full configuration (50 forward steps, then the adjoint with
checkpoints every 5 steps) giving forward and adjoint steps/s.  The other workloads of
the study (hex beam, tet block, tet beam, differentiation beam) are timed
after it.  Synthetic meshes; inputs are resident in HBM before the timed
region.

A step is one pass of the whole hot path: element assembly into A and b,
the refresh bookkeeping of the factor, preconditioned CG, and the update.
Warmup steps run the deterministic schedule so that a first factor is
installed; the timed steps run the asynchronous schedule.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
_T0 = time.perf_counter()


def _log(msg):
    """A progress line on stderr with the seconds since the start."""
    print(f"{msg} [{time.perf_counter() - _T0:.0f} s]", file=sys.stderr, flush=True)

HEADLINE = "hex_block"
# initial guess of the timed steps' CG: the A-norm projection onto the last
# 8 accelerations (x0 = 0 is timed beside it)
HEADLINE_WARM = 8
# the stale factor rotated to the current state (P^-1 = Q A_t0^-1 Q^T, per-node
# rotations); the plain stale factor is timed beside it
HEADLINE_ROTATE = 1


def _free(sim):
    import torch
    sim.ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _timed_run(w, prec, steps, warmup, timing=False, gpu_factor=True, warm_start=0, rotate=0):
    import torch

    from paper_2306_05893_amd import FE_FACTOR_ASYNC, FE_FACTOR_DETERMINISTIC
    from paper_2306_05893_amd.sim import Simulation

    sim = Simulation(w, prec=prec, device="cuda", factor_on_gpu=gpu_factor)
    det = sim.opts(rel_tol=1e-8, max_it=3000, refresh=w.refresh, lag=0,
                   mode=FE_FACTOR_DETERMINISTIC, warm_start=warm_start, rotate=rotate)
    asy = sim.opts(rel_tol=1e-8, max_it=3000, refresh=w.refresh, lag=0, mode=FE_FACTOR_ASYNC,
                   warm_start=warm_start, rotate=rotate)
    for _ in range(warmup):
        sim.step(det)
    torch.cuda.synchronize()
    if timing:
        sim.ctx.set_kernel_timing(True)
        sim.ctx.kernel_times()  # reset counters
    its, lags = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        st = sim.step(asy)
        its.append(st.solve.iterations)
        lags.append(st.factor_lag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = sim.ctx.kernel_times() if timing else None
    if timing:
        sim.ctx.set_kernel_timing(False)
    return {
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "steps_per_s": steps / (t1 - t0),
        "cg_it_mean": sum(its) / len(its),
        "cg_it_max": max(its),
        "factor_lag_mean": sum(lags) / len(lags),
        "kernels": kt,
        "sim": sim,
    }


def _leg(r):
    """The figures of one timed run, rounded for the JSON line."""
    return {"steps_per_s": round(r["steps_per_s"], 3), "ms_per_step": round(r["ms_per_step"], 3),
            "cg_it_mean": round(r["cg_it_mean"], 2), "cg_it_max": r["cg_it_max"],
            "factor_lag_mean": round(r["factor_lag_mean"], 1)}


# kernel names as rocprofv3 reports them.  The sweeps are named by family:
# their tile extents are chosen per level (forward k_tri_fwd<float, 64 or 128,
# true>, backward k_tri_bwd<float, 256 or 512, true>; the third argument: the
# panels of the hex block and the hex beam are read non-temporally, both
# factors being larger than the last-level cache), and a sweep's figures are
# averages over all its level launches.
KERNEL_SYMBOL = {"trisolve_fwd": "k_tri_fwd", "trisolve_bwd": "k_tri_bwd",
                 "spmv": "k_spmv<float, 16>", "element": "k_elem_hex<float, 1, true>"}


def _traffic_record(workload):
    return os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}_mixed.txt")


def _kernel_profile(sim, n_apply=40, n_spmv=40, n_assemble=10):
    """HIP-event durations of the preconditioner sweeps, SpMV and element
    kernels on a context whose factor is installed (events recorded on the
    launch stream around every launch; eager launches of the same kernels,
    each doing its full work)."""
    import torch
    ctx = sim.ctx
    A, _ = ctx.assemble(sim.params, sim.q, sim.v)
    r = torch.randn(ctx.sizes.n_dofs, dtype=torch.float64, device="cuda")
    z = ctx.precond_apply(r, A)
    torch.cuda.synchronize()
    ctx.set_kernel_timing(True)
    ctx.kernel_times()
    for _ in range(n_apply):
        ctx.precond_apply(r, A, z)
    for _ in range(n_spmv):
        ctx.spmv(A, r, z)
    for _ in range(n_assemble):
        ctx.assemble(sim.params, sim.q, sim.v, A)
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_kernel_timing(False)
    return kt


def _kernel_table(kt):
    kern = {}
    for name, d in kt.items():
        if d["count"]:
            gbs = d["bytes"] / (d["ms"] * 1e-3) / 1e9
            kern[name] = {"launches": d["count"], "avg_us": round(1e3 * d["ms"] / d["count"], 2),
                          "total_ms": round(d["ms"], 3), "GBps": round(gbs, 1),
                          "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    return kern


def _roofline(kt, workload):
    """Roofline entry of the dominant kernel (the sweep family with the larger
    total time): algorithmic bytes per launch over the average HIP-event
    launch duration."""
    dominant = max(("trisolve_fwd", "trisolve_bwd"), key=lambda n: kt[n]["ms"])
    dk = kt[dominant]
    achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": KERNEL_SYMBOL[dominant], "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _recorded_traffic(workload, KERNEL_SYMBOL[dominant]),
            "bytes_per_launch": dk["bytes"] / dk["count"],
            "avg_launch_us": 1e3 * dk["ms"] / dk["count"]}


def _recorded_traffic(workload, symbol):
    """HBM bytes per launch from the committed PMC record, or None when a
    source it depends on (the kernels, the tile schedule) has changed since
    the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(_traffic_record(workload)))
        if sorted(rec["sources_sha256"]) != sorted(TRAFFIC_SOURCES):
            return None
        for path, digest in rec["sources_sha256"].items():
            if hashlib.sha256(open(os.path.join(ROOT, path), "rb").read()).hexdigest() != digest:
                return None
        return round(rec["kernels"][symbol]["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _kernel_pass_only(workload, n_apply):
    """The event-timed kernel pass alone, on a context whose factor is that of
    the assembled workload at rest: no CG iterations run, so a kernel trace of
    this command holds the same sweep, SpMV and assembly launches as the
    events (plus one untimed preconditioner application first)."""
    import torch

    import synth
    from paper_2306_05893_amd import FE_PREC_MIXED
    from paper_2306_05893_amd.sim import Simulation

    w = synth.make(workload)
    sim = Simulation(w, prec=FE_PREC_MIXED, device="cuda", factor_on_gpu=True)
    A, _ = sim.ctx.assemble(sim.params, sim.q, sim.v)
    sim.ctx.factorize_now(A, 0)
    torch.cuda.synchronize()
    kt = _kernel_profile(sim, n_apply=n_apply, n_spmv=n_apply, n_assemble=min(10, n_apply))
    _free(sim)
    print(json.dumps({"workload": workload, "kernels": _kernel_table(kt),
                      "roofline": _roofline(kt, workload)}))


def _adjoint_leg(w, prec, nsteps, k, warm_start=0, rotate=0):
    """The full differentiable configuration: a target rollout with the
    second E field, then a rollout of nsteps forward steps with checkpoints
    every k steps (timed: forward steps/s) and its adjoint (timed: reverse
    steps/s, segment recomputation included); loss ||q_T - q_target||^2.
    The workload's tolerance and refresh period, asynchronous schedule, first
    factor of A at rest."""
    import torch

    from paper_2306_05893_amd import FE_FACTOR_ASYNC
    from paper_2306_05893_amd.sim import Simulation, rollout

    sim = Simulation(w, prec=prec, device="cuda", factor_on_gpu=True)
    A, _ = sim.ctx.assemble(sim.params, sim.q, sim.v)
    sim.ctx.factorize_now(A, 0)
    opts = sim.opts(rel_tol=w.rel_tol, max_it=3000, refresh=w.refresh, lag=0,
                    mode=FE_FACTOR_ASYNC, warm_start=warm_start, rotate=rotate)
    q0, v0 = sim.q.clone(), sim.v.clone()
    E_t = torch.as_tensor(w.extra["E_target"], dtype=torch.float64, device="cuda")
    with torch.no_grad():
        q_target, _ = rollout(E_t, q0, v0, sim.ctx, sim.params, nsteps, k, opts)
    sim.ctx.reset()
    sim.ctx.factorize_now(A, 0)
    E = sim.params.E.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qT, _ = rollout(E, q0, v0, sim.ctx, sim.params, nsteps, k, opts)
    loss = ((qT - q_target) ** 2).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ok = bool(torch.isfinite(E.grad).all())
    _free(sim)
    return {"forward_steps": nsteps, "checkpoint_every": k,
            "forward_steps_per_s": round(nsteps / (t1 - t0), 3),
            "adjoint_steps_per_s": round(nsteps / (t2 - t1), 3),
            "adjoint_s": round(t2 - t1, 2), "gradient_finite": ok}


def _headline(steps, warmup, extras, kernel_applies):
    """The headline workload: mixed steps/s (the value), the kernel pass that
    gives the roofline, and unless disabled the FP64 leg and the full
    forward + adjoint configuration."""
    import synth
    from paper_2306_05893_amd import FE_PREC_FP64, FE_PREC_MIXED

    w = synth.make(HEADLINE)
    _log(f"[bench] {HEADLINE}: {w.n_dofs} DOFs, {w.n_elems} elements")
    mixed = _timed_run(w, FE_PREC_MIXED, steps, warmup, warm_start=HEADLINE_WARM,
                       rotate=HEADLINE_ROTATE)
    _log(f"[bench] {HEADLINE} mixed {mixed['steps_per_s']:.2f} steps/s "
          f"it={mixed['cg_it_mean']:.1f} lag={mixed['factor_lag_mean']:.1f}")
    sizes = mixed["sim"].ctx.sizes
    kt = _kernel_profile(mixed["sim"], n_apply=kernel_applies, n_spmv=4 * kernel_applies,
                         n_assemble=kernel_applies)
    _free(mixed.pop("sim"))
    out = {"w": w, "mixed": mixed, "sizes": sizes, "kt": kt}
    if extras:
        fp64 = _timed_run(w, FE_PREC_FP64, steps, warmup, warm_start=HEADLINE_WARM,
                          rotate=HEADLINE_ROTATE)
        _free(fp64.pop("sim"))
        out["fp64"] = fp64
        _log(f"[bench] {HEADLINE} fp64 {fp64['steps_per_s']:.2f} steps/s "
              f"it={fp64['cg_it_mean']:.1f}")
        zero = _timed_run(w, FE_PREC_MIXED, steps, warmup, warm_start=0, rotate=0)
        _free(zero.pop("sim"))
        out["mixed_x0_zero"] = zero
        _log(f"[bench] {HEADLINE} mixed, plain stale factor, x0 = 0: "
             f"{zero['steps_per_s']:.2f} steps/s "
              f"it={zero['cg_it_mean']:.1f}")
        adj = _adjoint_leg(w, FE_PREC_MIXED, w.steps, w.extra["checkpoint_every"],
                           warm_start=HEADLINE_WARM, rotate=HEADLINE_ROTATE)
        out["adjoint"] = adj
        _log(f"[bench] {HEADLINE} {w.steps} forward steps {adj['forward_steps_per_s']} steps/s, "
              f"adjoint {adj['adjoint_steps_per_s']} steps/s")
    return out


def _other_workloads(steps, warmup):
    """The other GPU workloads of the study.  hex beam (107,163 DOFs): StVK
    and neo-Hookean, mixed and FP64 (refresh 10); the host-thread
    factorisation over a window long enough for its factors to land; the CG
    warm start.  tet block (206,763 DOFs): mixed and FP64 (refresh 10).  tet
    beam (1,275 DOFs): FP64, exact factor every step, rel-res 1e-10.
    differentiation beam (14,883 DOFs): FP64 forward and adjoint steps/s."""
    import dataclasses

    import synth
    from paper_2306_05893_amd import (FE_FACTOR_DETERMINISTIC, FE_NEO_HOOKEAN, FE_PREC_FP64,
                                      FE_PREC_MIXED)
    from paper_2306_05893_amd.sim import Simulation

    out = {}
    hb = synth.make("hex_beam")
    rec = {"n_dofs": hb.n_dofs, "refresh": hb.refresh, "steps": steps}
    for tag, w, prec in (("stvk_mixed", hb, FE_PREC_MIXED), ("stvk_fp64", hb, FE_PREC_FP64),
                         ("nh_mixed", dataclasses.replace(hb, material=FE_NEO_HOOKEAN),
                          FE_PREC_MIXED),
                         ("nh_fp64", dataclasses.replace(hb, material=FE_NEO_HOOKEAN),
                          FE_PREC_FP64)):
        r = _timed_run(w, prec, steps, warmup)
        _free(r.pop("sim"))
        rec[tag] = _leg(r)
    long_steps = max(steps, 150)
    r = _timed_run(hb, FE_PREC_MIXED, long_steps, warmup, gpu_factor=False)
    _free(r.pop("sim"))
    rec["stvk_mixed_host_factor"] = dict(_leg(r), steps=long_steps)
    r = _timed_run(hb, FE_PREC_MIXED, steps, warmup, warm_start=1)
    _free(r.pop("sim"))
    rec["stvk_mixed_warm_start"] = _leg(r)
    out["hex_beam"] = rec
    _log(f"[bench] hex_beam StVK mixed {rec['stvk_mixed']['steps_per_s']} / fp64 "
         f"{rec['stvk_fp64']['steps_per_s']}, NH mixed {rec['nh_mixed']['steps_per_s']} steps/s")
    w = synth.make("tet_block")
    rec = {"n_dofs": w.n_dofs, "refresh": w.refresh, "steps": steps}
    for tag, prec in (("mixed", FE_PREC_MIXED), ("fp64", FE_PREC_FP64)):
        r = _timed_run(w, prec, steps, warmup)
        _free(r.pop("sim"))
        rec[tag] = _leg(r)
    out["tet_block"] = rec
    _log(f"[bench] tet_block mixed {rec['mixed']['steps_per_s']} / fp64 "
          f"{rec['fp64']['steps_per_s']} steps/s")
    # tet beam: its own 10 steps, exact factor each step (refresh 1, lag 0)
    import torch
    w = synth.make("tet_beam")
    sim = Simulation(w, prec=FE_PREC_FP64, device="cuda", factor_on_gpu=True)
    det = sim.opts(rel_tol=1e-10, max_it=500, refresh=1, lag=0, mode=FE_FACTOR_DETERMINISTIC)
    sim.step(det)
    sim.ctx.reset()
    sim.q.copy_(torch.as_tensor(w.q0(), device="cuda"))
    sim.v.zero_()
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for _ in range(w.steps):
        its.append(sim.step(det).solve.iterations)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _free(sim)
    out["tet_beam"] = {"n_dofs": w.n_dofs, "steps": w.steps, "prec": "fp64",
                       "steps_per_s": round(w.steps / dt, 2), "cg_it_mean": sum(its) / len(its)}
    w = synth.make("hex_diff")
    out["hex_diff"] = dict({"n_dofs": w.n_dofs, "prec": "fp64"},
                           **_adjoint_leg(w, FE_PREC_FP64, w.steps, w.extra["checkpoint_every"]))
    _log(f"[bench] tet_beam {out['tet_beam']['steps_per_s']} steps/s; hex_diff forward "
          f"{out['hex_diff']['forward_steps_per_s']} / adjoint "
          f"{out['hex_diff']['adjoint_steps_per_s']} steps/s")
    return out


def _materials(steps=30, warmup=10):
    """The paper's other element models on the benchmark workload (Sec. 3.1:
    co-rotational and Mooney-Rivlin): mixed steps/s on the same schedule and
    the duration of one assembly (element kernel + gather)."""
    import dataclasses

    import synth
    from paper_2306_05893_amd import FE_COROTATIONAL, FE_MOONEY_RIVLIN, FE_PREC_MIXED

    out = {}
    for name, mat in (("corotational", FE_COROTATIONAL), ("mooney_rivlin", FE_MOONEY_RIVLIN)):
        w = dataclasses.replace(synth.make("hex_beam"), material=mat)
        r = _timed_run(w, FE_PREC_MIXED, steps, warmup)
        kt = _kernel_profile(r["sim"], n_apply=0, n_spmv=0, n_assemble=10)
        r["sim"].ctx.close()
        el = kt["element"]
        out[name] = {"steps_per_s": round(r["steps_per_s"], 2),
                     "cg_it_mean": round(r["cg_it_mean"], 2),
                     "factor_lag_mean": round(r["factor_lag_mean"], 1),
                     "assembly_us": round(1e3 * el["ms"] / max(el["count"], 1), 1)}
        _log(f"[bench] {name}: {out[name]['steps_per_s']} steps/s, assembly "
              f"{out[name]['assembly_us']} us")
    return out


def _topology():
    """Full assembly on a topology change (Sec. 4.2) on the hex beam: the
    keepStruct test on the GPU when nothing changed, and the rebuild of
    pattern, map, ordering, factor structure and device workspace after a cut
    (one layer of 400 elements removed; host work plus the upload), followed
    by the first assembly on the new context."""
    import torch

    import synth
    from paper_2306_05893_amd import FE_PREC_MIXED
    from paper_2306_05893_amd.sim import Simulation

    w = synth.make("hex_beam")
    sim = Simulation(w, prec=FE_PREC_MIXED, device="cuda", factor_on_gpu=True)
    sim.ctx.assemble(sim.params, sim.q, sim.v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        assert sim.set_topology(w.conn, w.E) is False
    t_keep = (time.perf_counter() - t0) / 10
    zc = w.X[w.conn][:, :, 2].mean(axis=1) / w.spacing
    keep = ~((zc >= 40) & (zc < 41))
    t0 = time.perf_counter()
    assert sim.set_topology(w.conn[keep], w.E[keep]) is True
    sim.ctx.assemble(sim.params, sim.q, sim.v)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    out = {"keepstruct_check_ms": round(1e3 * t_keep, 3), "full_assembly_ms": round(1e3 * t_full, 1),
           "elements_removed": int((~keep).sum()), "nnz_after": int(sim.ctx.sizes.nnz)}
    sim.ctx.close()
    _log(f"[bench] topology: keepStruct check {out['keepstruct_check_ms']} ms, full assembly "
          f"{out['full_assembly_ms']} ms")
    return out


MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}


def _contact(k=246, n_rep=10, pgs_sweeps=100):
    """Contact through Lagrange multipliers on the hex beam (paper Sec. 6.2;
    its liver scene averages 246 constraints per step): the compliance matrix
    W = H P^{-1} H^T built with the many-right-hand-side sweeps, against the
    same W from k single-right-hand-side preconditioner applications; the
    projected Gauss-Seidel solve; one whole three-stage contact solve.  Mixed
    precision (FP32 MFMA sweeps) and FP64 (FP64 MFMA)."""
    import numpy as np
    import torch

    import synth
    from paper_2306_05893_amd import FE_PREC_FP64, FE_PREC_MIXED
    from paper_2306_05893_amd.sim import Constraints, Simulation

    w = synth.make("hex_beam")
    Hh, d0 = synth.contact_constraints(w, k, 31)
    out = {"workload": f"hex_beam (107163 DOFs), {k} contact constraints on the y = min face "
                       "(alternating node-on-plane and point-on-triangle rows)", "k": k}
    for tag, prec in (("mixed", FE_PREC_MIXED), ("fp64", FE_PREC_FP64)):
        sim = Simulation(w, prec=prec, device="cuda", factor_on_gpu=True)
        ctx = sim.ctx
        A, b = ctx.assemble(sim.params, sim.q, sim.v)
        ctx.factorize_now(A, 0)
        H = Constraints.from_host(Hh, "cuda")
        W = ctx.compliance(H)                      # warm-up (workspace, code objects)
        torch.cuda.synchronize()
        ms = []
        for _ in range(n_rep):
            t0 = time.perf_counter()
            ctx.compliance(H, W=W)                 # synchronises
            ms.append(1e3 * (time.perf_counter() - t0))
        ms.sort()
        # kernel-level figures of the many-right-hand-side sweeps (HIP events
        # around every launch, separate pass)
        ctx.set_kernel_timing(True)
        ctx.kernel_times()
        for _ in range(3):
            ctx.compliance(H, W=W)
        kt = ctx.kernel_times()
        ctx.set_kernel_timing(False)
        # the same W from k single applications (columns of H^T one by one)
        HT = torch.zeros(w.n_dofs, k, dtype=torch.float64, device="cuda")
        rp, col, val = Hh
        for a in range(k):
            HT[torch.as_tensor(col[rp[a]:rp[a + 1]].astype(np.int64), device="cuda"), a] = \
                torch.as_tensor(val[rp[a]:rp[a + 1]], device="cuda")
        cols = [HT[:, a].contiguous() for a in range(k)]
        z = torch.empty(w.n_dofs, dtype=torch.float64, device="cuda")
        ctx.precond_apply(cols[0], z=z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a in range(k):
            ctx.precond_apply(cols[a], z=z)
        torch.cuda.synchronize()
        single_ms = 1e3 * (time.perf_counter() - t0)
        # projected Gauss-Seidel, fixed sweep count
        c = ctx.constraint_apply(H, sim.q, s_h=1.0)
        lam, info = ctx.pgs(W, c, max_sweeps=pgs_sweeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, info = ctx.pgs(W, c, max_sweeps=pgs_sweeps)
        torch.cuda.synchronize()
        pgs_ms = 1e3 * (time.perf_counter() - t0)
        # whole contact solve: free PCG, compliance, PGS, correction PCG
        x_free, _ = ctx.pcg_solve(A, b, rel_tol=1e-8, max_it=500)
        hx = ctx.constraint_apply(H, x_free).cpu().numpy()
        delta = torch.as_tensor(hx - np.abs(hx).max() * 0.5 * d0, device="cuda")
        ctx.contact_solve(A, b, H, delta, sweeps=pgs_sweeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, _, lam, _, st = ctx.contact_solve(A, b, H, delta, sweeps=pgs_sweeps)
        torch.cuda.synchronize()
        solve_ms = 1e3 * (time.perf_counter() - t0)
        dt = "f32" if prec == FE_PREC_MIXED else "f64"
        kern = {}
        for name in ("multi_fwd", "multi_bwd"):
            d = kt[name]
            tf = d["bytes"] / (d["ms"] * 1e-3) / 1e12
            kern[name] = {"launches": d["count"], "avg_us": round(1e3 * d["ms"] / d["count"], 2),
                          "TFLOPs": round(tf, 2),
                          "frac_mfma_peak": round(tf / MFMA_PEAK_TFLOPS[dt], 4)}
        tot_ms = kt["multi_fwd"]["ms"] + kt["multi_bwd"]["ms"]
        tot_fl = kt["multi_fwd"]["bytes"] + kt["multi_bwd"]["bytes"]
        out[tag] = {"compliance_ms_median": round(ms[len(ms) // 2], 3),
                    "compliance_ms_min": round(ms[0], 3),
                    "single_rhs_applies_ms": round(single_ms, 3),
                    "speedup_vs_single_rhs": round(single_ms / ms[len(ms) // 2], 2),
                    "sweeps_TFLOPs": round(tot_fl / (tot_ms * 1e-3) / 1e12, 2),
                    "sweeps_frac_mfma_peak": round(tot_fl / (tot_ms * 1e-3) / 1e12
                                                   / MFMA_PEAK_TFLOPS[dt], 4),
                    "mfma_dtype": dt, "kernels": kern,
                    "pgs_ms": round(pgs_ms, 3), "pgs_sweeps": int(info[0]),
                    "contact_solve_ms": round(solve_ms, 3),
                    "contact_active": int((lam > 0).sum()),
                    "cg_it_free_correction": [st["free"].iterations,
                                              st["correction"].iterations]}
        _log(f"[bench] contact {tag}: W in {out[tag]['compliance_ms_median']} ms "
              f"({out[tag]['speedup_vs_single_rhs']}x vs single applies), sweeps "
              f"{out[tag]['sweeps_TFLOPs']} TFLOP/s")
        ctx.close()
    return out


def _factor_only(workload, n=5):
    """Standalone GPU refactorisations of a workload's A at rest (mixed
    precision, FP64 factor), timed one by one: the input of the factorisation
    kernel profile."""
    import torch

    import synth
    from paper_2306_05893_amd import FE_PREC_MIXED
    from paper_2306_05893_amd.sim import Simulation

    w = synth.make(workload)
    sim = Simulation(w, prec=FE_PREC_MIXED, device="cuda", factor_on_gpu=True)
    A, _ = sim.ctx.assemble(sim.params, sim.q, sim.v)
    ms = []
    for k in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.ctx.factorize_now(A, k)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
    s = sim.ctx.sizes
    sim.ctx.close()
    print(json.dumps({"workload": workload, "factor_ms": [round(x, 3) for x in ms],
                      "factor_flops": s.factor_flops, "factor_lower_entries": int(s.factor_lower)}))




def _age_curve(workload, nsteps, variants):
    """CG iterations against the age of the factor, along the workload's own
    trajectory: deterministic schedule with the workload's refresh period and
    lag 0, so step kR + j solves with the factor of A_{kR} (age j).  One run
    per variant (precision, warm start); per step: age, iterations, and the
    wall time of the step (the blocking factorisation at each refresh is
    included in that step's time)."""
    import torch

    import synth
    from paper_2306_05893_amd import FE_FACTOR_DETERMINISTIC, FE_PREC_FP64, FE_PREC_MIXED
    from paper_2306_05893_amd.sim import Simulation

    w = synth.make(workload)
    out = {"workload": workload, "n_dofs": w.n_dofs, "refresh": w.refresh, "steps": nsteps,
           "variants": {}}
    for tag in variants:
        prec = FE_PREC_FP64 if tag.startswith("fp64") else FE_PREC_MIXED
        warm = 1 if "warm" in tag else (int(tag.split("proj")[1][:1]) if "proj" in tag else 0)
        rot = 1 if tag.endswith("rot") else 0
        sim = Simulation(w, prec=prec, device="cuda", factor_on_gpu=True)
        det = sim.opts(rel_tol=1e-8, max_it=3000, refresh=w.refresh, lag=0,
                       mode=FE_FACTOR_DETERMINISTIC, warm_start=warm, rotate=rot)
        ages, its, ms = [], [], []
        for k in range(nsteps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = sim.step(det)
            torch.cuda.synchronize()
            ms.append(round(1e3 * (time.perf_counter() - t0), 2))
            ages.append(int(st.factor_lag))
            its.append(int(st.solve.iterations))
        _free(sim)
        by_age = {}
        for a, i in zip(ages, its):
            by_age.setdefault(a, []).append(i)
        out["variants"][tag] = {"age": ages, "iterations": its, "step_ms": ms,
                                "mean_iterations_by_age": {a: round(sum(v) / len(v), 2)
                                                           for a, v in sorted(by_age.items())}}
        _log(f"[bench] age curve {tag}: mean iterations {sum(its) / len(its):.1f}")
    print(json.dumps(out))


def _host_cores():
    """Cores this process may run on (what `nproc` reports) and the thread
    count the oracle's BLAS calls are given (capped by OMP_NUM_THREADS when
    set, as on a shared host)."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(nproc, int(env)) if env.isdigit() and int(env) > 0 else nproc
    return nproc, threads


def _cpu_child(mode, threads, timeout=900):
    env = dict(os.environ, OPENBLAS_NUM_THREADS=str(threads), OMP_NUM_THREADS=str(threads),
               MKL_NUM_THREADS=str(threads))
    p = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", mode],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env,
                       timeout=timeout)
    if p.returncode != 0:
        raise RuntimeError(p.stderr[-400:])
    return json.loads(p.stdout.strip().splitlines()[-1])


SLAB_LAYERS = 12   # cell layers of the hex block in the CPU sample (1/16 of 192)


def _cpu_baseline(small_configs=False):
    """The FP64 oracle on the GPU machine's host cores.

    Headline workload (value): a bounded sample, the bottom 12 of the 192
    cell layers of the hex block (1/16 of its elements and nonzeros, same
    material field, z = 0 face fixed): one oracle step from rest, i.e. numpy
    element tangents and forces, triplet-sort assembly through the map, and
    an FP64 Jacobi-PCG solve capped in time, plus one CSR SpMV; every phase
    is scaled x16 to the full block.  The capped solve does not converge, so
    the figure is an upper bound on the oracle's steps/s.  With
    small_configs (``--cpu-phases``), the small configurations run whole
    (tet beam 10 steps with dense Cholesky, differentiation beam 20 steps with
    banded Cholesky), with one BLAS thread and with all the cores."""
    nproc, threads = _host_cores()
    try:
        s = _cpu_child("slab", threads)
    except (RuntimeError, subprocess.TimeoutExpired) as e:
        return {"value": None, "unit": "steps/s", "cores": threads, "nproc": nproc,
                "kind": "oracle", "sample": f"failed: {e}"}
    scale = s["scale"]
    t_step = scale * (s["t_assemble"] + s["t_pcg"]) + s["t_update_full"]
    out = {"value": round(1.0 / t_step, 5), "unit": "steps/s", "cores": threads, "nproc": nproc,
           "kind": "oracle",
           "sample": (f"hex block, bottom {SLAB_LAYERS} of 192 cell layers ({s['n_elems']} HEX8, "
                      f"{s['n_dofs']} DOFs, 1/{scale:g} of the block): one oracle step from rest, "
                      f"element tangents + triplet-sort assembly {s['t_assemble']:.1f} s, FP64 "
                      f"Jacobi-PCG stopped after {s['t_pcg']:.1f} s ({s['pcg_it']} iterations, "
                      f"rel-res {s['pcg_res']:.1e}, not converged); phases scaled x{scale:g}; an "
                      f"upper bound on the oracle's steps/s (BLAS threads {threads} of nproc "
                      f"{nproc}; the numpy element and CSR code runs on one thread)"),
           "phases_full_size_s": {"assembly": round(scale * s["t_assemble"], 2),
                                  "csr_spmv": round(scale * s["t_spmv"], 3),
                                  "jacobi_pcg_iteration": round(scale * s["t_pcg"] /
                                                                max(s["pcg_it"], 1), 3),
                                  "pattern_once": round(scale * s["t_pattern"], 1)}}
    if not small_configs:
        return out
    small = {}
    for tag, th in (("1_thread", 1), (f"{threads}_threads", threads)):
        try:
            small[tag] = _cpu_child("small", th)
        except (RuntimeError, subprocess.TimeoutExpired) as e:
            small[tag] = {"failed": str(e)[-200:]}
    out["small_configs"] = small
    return out


def _cpu_phases():
    """The oracle's per-phase times at full size (hex beam, tet block) and the
    headline's CPU baseline, one JSON line; no GPU is touched."""
    nproc, threads = _host_cores()
    out = {"nproc": nproc, "threads": threads, "phases": {}}
    for name in ("hex_beam", "tet_block"):
        try:
            out["phases"][name] = _cpu_child(f"phases:{name}", threads)
        except (RuntimeError, subprocess.TimeoutExpired) as e:
            out["phases"][name] = {"failed": str(e)[-200:]}
        _log(f"[bench] oracle phases {name}: {out['phases'][name]}")
    out["headline"] = _cpu_baseline(small_configs=True)
    print(json.dumps(out))


def _cpu_baseline_child(mode):
    import dataclasses

    import numpy as np

    import synth
    from oracle import assembly, solve
    from oracle import step as ostep
    if mode == "slab":
        w = synth.make(HEADLINE)
        nx, ny, nz = w.dims
        n_nodes = (nx + 1) * (ny + 1) * (SLAB_LAYERS + 1)
        n_el = nx * ny * SLAB_LAYERS
        # elements and nodes are numbered with z slowest, so the bottom
        # layers are leading ranges of both
        assert int(w.conn[:n_el].max()) < n_nodes
        sub = dataclasses.replace(w, X=w.X[:n_nodes], conn=np.ascontiguousarray(w.conn[:n_el]),
                                  E=w.E[:n_el], fixed=w.fixed[:3 * n_nodes],
                                  f_nodal=w.f_nodal[:n_nodes])
        t0 = time.perf_counter()
        pat = ostep.pattern(sub)
        t1 = time.perf_counter()
        q, v = sub.q0(), sub.v0()
        s = ostep.assemble(sub, q, v, pat=pat)
        t2 = time.perf_counter()
        y = assembly.csr_matvec(pat.row_ptr, pat.col_idx, s.vals, s.b)
        t3 = time.perf_counter()
        a, it, res = solve.jacobi_pcg(pat.row_ptr, pat.col_idx, s.vals, s.b, rel_tol=1e-8,
                                      time_limit=10.0)
        t4 = time.perf_counter()
        qf, vf, af = w.q0(), w.v0(), np.zeros(w.n_dofs)
        t5 = time.perf_counter()
        v1 = vf + w.h * af
        q1 = qf + w.h * v1
        t6 = time.perf_counter()
        assert np.isfinite(y).all() and np.isfinite(a).all() and np.isfinite(q1).all()
        print(json.dumps({"n_elems": n_el, "n_dofs": sub.n_dofs, "scale": w.n_elems / n_el,
                          "t_pattern": t1 - t0, "t_assemble": t2 - t1, "t_spmv": t3 - t2,
                          "t_pcg": t4 - t3, "pcg_it": int(it), "pcg_res": float(res),
                          "t_update_full": t6 - t5}))
        return
    if mode.startswith("phases:"):
        # one oracle step from rest at full size, phase by phase
        w = synth.make(mode.split(":", 1)[1])
        t0 = time.perf_counter()
        pat = ostep.pattern(w)
        t1 = time.perf_counter()
        s = ostep.assemble(w, w.q0(), w.v0(), pat=pat)
        t2 = time.perf_counter()
        y = assembly.csr_matvec(pat.row_ptr, pat.col_idx, s.vals, s.b)
        t3 = time.perf_counter()
        a, it, res = solve.jacobi_pcg(pat.row_ptr, pat.col_idx, s.vals, s.b, rel_tol=1e-8,
                                      time_limit=20.0)
        t4 = time.perf_counter()
        assert np.isfinite(y).all() and np.isfinite(a).all()
        print(json.dumps({"workload": w.name, "n_dofs": w.n_dofs, "nnz": int(pat.col_idx.size),
                          "pattern_s": round(t1 - t0, 3), "assembly_s": round(t2 - t1, 3),
                          "csr_spmv_s": round(t3 - t2, 4), "jacobi_pcg_s": round(t4 - t3, 2),
                          "jacobi_pcg_iterations": int(it), "jacobi_pcg_rel_res": float(res),
                          "jacobi_pcg_converged": bool(res <= 1e-8)}))
        return
    out = {}
    for name in ("tet_beam", "hex_diff"):
        w = synth.make(name)
        solver = ostep.default_solver(w.n_dofs)
        pat = ostep.pattern(w)
        q, v = w.q0(), w.v0()
        t0 = time.perf_counter()
        for _ in range(w.steps):
            q, v, _ = ostep.step(w, q, v, solver=solver, pat=pat)
        dt = time.perf_counter() - t0
        assert np.isfinite(q).all()
        out[name] = {"steps": w.steps, "solver": solver, "steps_per_s": round(w.steps / dt, 3)}
    print(json.dumps(out))


# sources whose change invalidates a recorded traffic figure: the sweep and
# SpMV kernels, and the analysis that lays out the sweep tiles
TRAFFIC_SOURCES = ("paper_2306_05893_amd/csrc/kernels_solve.hip",
                   "paper_2306_05893_amd/csrc/host_analyse.cpp")


def _write_traffic_record(fetch_csv, write_csv, workload, copy_mib):
    """Machine-readable HBM traffic of the SpMV and sweep kernels from two
    rocprofv3 counter runs of the kernel pass (FETCH_SIZE, then WRITE_SIZE,
    KiB per dispatch, with --calibrate-copy-mib): each counter is scaled by
    what it reads for the calibration copy of known size, and the sweeps are
    averaged per family over all their level launches (host only)."""
    import csv
    import hashlib
    import re

    def load(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            nm = re.sub(r"^void ", "", r["Kernel_Name"]).replace("fe::(anonymous namespace)::", "")
            nm = nm[:nm.index("(")] if "(" in nm else nm
            if nm.startswith("k_tri_fwd") or nm.startswith("k_tri_bwd"):
                nm = nm[:len("k_tri_fwd")]
            acc.setdefault(nm, []).append(float(r["Counter_Value"]))
        return acc

    f, w = load(fetch_csv, "FETCH_SIZE"), load(write_csv, "WRITE_SIZE")
    cal = [k for k in f if "elementwise" in k]
    if len(cal) != 1:
        raise SystemExit("the counter runs need exactly one calibration copy kernel")
    kib = copy_mib * 1024.0
    fs = kib / (sum(f[cal[0]]) / len(f[cal[0]]))
    ws = kib / (sum(w[cal[0]]) / len(w[cal[0]]))
    rec = {"workload": f"{workload} mixed (bench.py --kernel-pass-only --workload {workload} "
                       f"--kernel-applies 3 --calibrate-copy-mib {copy_mib})",
           "sources_sha256": {p: hashlib.sha256(open(os.path.join(ROOT, p), "rb").read())
                              .hexdigest() for p in TRAFFIC_SOURCES},
           "fetch_scale": fs, "write_scale": ws, "kernels": {}}
    for k in (KERNEL_SYMBOL["spmv"], KERNEL_SYMBOL["trisolve_fwd"], KERNEL_SYMBOL["trisolve_bwd"]):
        fb = sum(f[k]) / len(f[k]) * 1024 * fs
        wb = sum(w[k]) / len(w[k]) * 1024 * ws
        rec["kernels"][k] = {"dispatches": len(f[k]), "fetch_bytes_per_launch": fb,
                             "write_bytes_per_launch": wb, "traffic_bytes_per_launch": fb + wb}
    with open(_traffic_record(workload), "w") as out:
        json.dump(rec, out, indent=1)
    print(json.dumps({k: round(v["traffic_bytes_per_launch"] / 1e6, 1)
                      for k, v in rec["kernels"].items()}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline mixed leg only (no FP64/adjoint legs, no other workloads)")
    ap.add_argument("--cpu-baseline-child", default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-phases", action="store_true",
                    help="only time the oracle's phases (pattern, assembly, CSR SpMV, capped "
                         "Jacobi-PCG) at full size on the hex beam and the tet block, and the "
                         "CPU baseline of the headline, on the host cores (no GPU)")
    ap.add_argument("--factor-only", type=int, default=0, metavar="N",
                    help="only time N standalone GPU refactorisations of --workload")
    ap.add_argument("--workload", default=HEADLINE,
                    help="workload of --kernel-pass-only / --factor-only")
    ap.add_argument("--kernel-applies", type=int, default=5,
                    help="preconditioner applications in the event-timed kernel pass")
    ap.add_argument("--topology-only", action="store_true",
                    help="only time the keepStruct test and a full assembly after a cut")
    ap.add_argument("--materials-only", action="store_true",
                    help="only run the co-rotational and Mooney-Rivlin legs")
    ap.add_argument("--contact-only", action="store_true",
                    help="only run the contact measurements (compliance matrix, PGS)")
    ap.add_argument("--kernel-pass-only", action="store_true",
                    help="only the event-timed kernel pass (factor of A at rest)")
    ap.add_argument("--age-curve", type=int, default=0, metavar="STEPS",
                    help="only record CG iterations against factor age over STEPS steps of "
                         "--workload (deterministic schedule; mixed with x0 = 0, the previous "
                         "acceleration or the projection onto the last 8, and FP64 with x0 = 0)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (read + write), the "
                         "reference dispatch for scaling hardware byte counters")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="only write the traffic record of --workload from the counter "
                         "collections of two rocprofv3 runs of the kernel pass (FETCH_SIZE, "
                         "then WRITE_SIZE, both with --calibrate-copy-mib 1024); no GPU")
    args = ap.parse_args()
    if args.traffic_record:
        _write_traffic_record(args.traffic_record[0], args.traffic_record[1], args.workload, 1024)
        return
    if args.cpu_baseline_child:
        _cpu_baseline_child(args.cpu_baseline_child)
        return
    if args.cpu_phases:
        _cpu_phases()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is described in the design notes but not implemented.",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy_mib > 0:
        import torch
        nel = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)        # reads and writes nel * 4 bytes
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        _log(f"[bench] calibration copy {args.calibrate_copy_mib} MiB done")
    if args.factor_only > 0:
        _factor_only(args.workload, args.factor_only)
        return
    if args.age_curve > 0:
        _age_curve(args.workload, args.age_curve,
                   ("mixed", "mixed_rot", "mixed_proj8", "mixed_proj8_rot", "fp64"))
        return
    if args.kernel_pass_only:
        _kernel_pass_only(args.workload, args.kernel_applies)
        return
    if args.contact_only:
        print(json.dumps({"contact": _contact()}))
        return
    if args.materials_only:
        print(json.dumps({"materials": _materials()}))
        return
    if args.topology_only:
        print(json.dumps({"topology": _topology()}))
        return

    extras = not args.no_extras
    h = _headline(args.steps, args.warmup, extras, args.kernel_applies)
    w, mixed, sizes, kt = h["w"], h["mixed"], h["sizes"], h["kt"]
    kern = _kernel_table(kt)
    roofline = _roofline(kt, HEADLINE)
    line_extras = {}
    if extras:
        fp64 = h["fp64"]
        line_extras = {
            "fp64_steps_per_s": round(fp64["steps_per_s"], 3),
            "fp64_ms_per_step": round(fp64["ms_per_step"], 3),
            "fp64_cg_it_mean": round(fp64["cg_it_mean"], 2),
            "fp64_factor_lag_mean": round(fp64["factor_lag_mean"], 1),
            "mixed_vs_fp64": round(mixed["steps_per_s"] / fp64["steps_per_s"], 3),
            "mixed_plain_x0_zero": _leg(h["mixed_x0_zero"]),
            "adjoint_steps_per_s": h["adjoint"]["adjoint_steps_per_s"],
            "full_config": h["adjoint"],
        }
        line_extras["other_workloads"] = _other_workloads(args.steps, args.warmup)
        line_extras["contact"] = _contact()
        line_extras["materials"] = _materials()
        line_extras["topology"] = _topology()
    cpu = None if args.no_cpu_baseline else _cpu_baseline()
    line = {
        "metric": "implicit steps/s at rel-res 1e-8 (mixed precision; FP64 and adjoint "
                  "steps/s beside it)",
        "value": round(mixed["steps_per_s"], 3),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "hex_block 48x48x192 HEX8 two-material neo-Hookean (2000 / 20000 "
                               "Pa, 64 spherical inclusions of radius 4 cells), gravity, "
                               f"{w.n_dofs} DOFs, h=0.01, LDL^T refreshed every {w.refresh} "
                               "steps (asynchronous, FP64 factorisation on its own GPU "
                               "stream), mixed precision, rel-res 1e-8, CG initial guess "
                               f"projected on the last {HEADLINE_WARM} accelerations"
                               + (", stale factor rotated to the current state"
                                  if HEADLINE_ROTATE else ""),
                   "preconditioner": ("stale LDL^T rotated per node to the current state"
                                      if HEADLINE_ROTATE else "stale LDL^T"),
                   "cg_initial_guess": (f"A-norm projection on the last {HEADLINE_WARM} "
                                        "accelerations" if HEADLINE_WARM >= 2 else
                                        "previous acceleration" if HEADLINE_WARM == 1 else
                                        "zero"),
                   "n_dofs": w.n_dofs, "n_elems": w.n_elems, "nnz": int(sizes.nnz),
                   "factor_lower_entries": int(sizes.factor_lower),
                   "levels": int(sizes.n_levels), "refresh": w.refresh,
                   "cg_it_mean": round(mixed["cg_it_mean"], 2), "cg_it_max": mixed["cg_it_max"],
                   "factor_lag_mean": round(mixed["factor_lag_mean"], 1)},
        "spmv_GBps": kern.get("spmv", {}).get("GBps"),
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(line_extras)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
