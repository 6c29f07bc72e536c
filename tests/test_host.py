"""CPU tests of the library's host logic (no GPU needed).

* the shared library loads and exports every function include/fe.h declares;
* the CSR pattern and the triplet -> CSR map built by the library's two
  counting-sort transposes are bit-identical to the oracle's comparison sort;
* the nested-dissection ordering is a permutation with the fixed DOFs last;
* the host FP64 LDL^T in explicit-inverse panel form applies A^{-1} (checked
  against the oracle's dense Cholesky solve);
* bad input is rejected with FE_EINVAL.
"""
import ctypes as C
import itertools
import os
import re

import numpy as np
import pytest

import synth
from oracle import assembly, solve, step

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytest.importorskip("torch")
from paper_2306_05893_amd import _lib  # noqa: E402
from paper_2306_05893_amd.sim import FEContext  # noqa: E402


def _ctx(w, prec=0, leaf=0):
    return FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=prec, leaf_nodes=leaf, device="cpu")


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    header = open(os.path.join(ROOT, "include", "fe.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char \*)\s*(fe_\w+)\s*\(", header, re.M))
    assert {"fe_build_pattern", "fe_assemble", "fe_factor_async", "fe_pcg_solve", "fe_step",
            "fe_step_adjoint"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


@pytest.mark.parametrize("mesh", ["tiny_tet", "tiny_hex", "tet_beam", "hex_diff", "hex_beam",
                                  "tet_block"])
def test_pattern_and_map_bit_exact(mesh):
    w = synth.make(mesh)
    ctx = _ctx(w)
    rp, ci, mp = ctx.export_pattern()
    ro, co, tm, fd, ds = assembly.build_pattern(w.n_dofs, w.conn, w.fixed)
    assert np.array_equal(rp, ro)
    assert np.array_equal(ci, co)
    assert np.array_equal(mp, tm)
    assert ctx.sizes.compact_map == 1
    assert ctx.sizes.nnz == co.size
    assert ctx.sizes.map_len == tm.size


def _hex_blocks(n):
    """Node blocks of the trilinear-hex grid with n[i] nodes per axis: node
    pairs within one cell, i.e. offsets in {-1, 0, 1} per axis."""
    return int(np.prod([3 * k - 2 for k in n]))


def _kuhn_blocks(n):
    """Node blocks of the Kuhn (Freudenthal) tet grid: the node itself plus
    both directions of every edge; the edges run along the seven offsets
    d in {0, 1}^3 minus 0, each present prod(n_i - d_i) times."""
    s = sum(int(np.prod([k - di for k, di in zip(n, d)]))
            for d in itertools.product((0, 1), repeat=3) if any(d))
    return int(np.prod(n)) + 2 * s


@pytest.mark.parametrize("mesh", ["hex_beam", "tet_block", "hex_block"])
def test_nnz_matches_closed_form_block_counts(mesh):
    """Structural nonzeros at full size against closed forms of the grid: with
    no fixed DOF, 9 per node block of the whole grid; with the z = 0 face fixed,
    9 per node block of the free sub-grid (the nodes above z = 0) plus one
    diagonal entry per fixed DOF."""
    w = synth.make(mesh)
    n = [d + 1 for d in w.dims]
    blocks = _hex_blocks if w.elem_type == 8 else _kuhn_blocks
    ctx = FEContext(w.X, w.conn, w.elem_type, None, device="cpu")
    assert ctx.sizes.nnz == 9 * blocks(n)
    ctx.close()
    n_fixed = int(w.fixed.sum())
    assert n_fixed == 3 * n[0] * n[1]
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, device="cpu")
    assert ctx.sizes.nnz == 9 * blocks([n[0], n[1], n[2] - 1]) + n_fixed
    print(f"{mesh}: nnz {ctx.sizes.nnz} ({blocks(n)} node blocks without constraints)")
    ctx.close()


def test_pattern_per_dof_constraints_fall_back_to_int32_map():
    """Roller constraints (some DOFs of a node fixed) still give the exact
    pattern and map; the 1-byte node-slot map is not used."""
    w = synth.make("tiny_hex")
    fixed = np.zeros(w.n_dofs, dtype=np.uint8)
    fixed[2::3][np.abs(w.X[:, 2]) < 1e-12] = 1   # z-DOF of the z = 0 face
    fixed[0] = fixed[1] = 1
    w.fixed = fixed
    ctx = _ctx(w)
    rp, ci, mp = ctx.export_pattern()
    ro, co, tm, _, _ = assembly.build_pattern(w.n_dofs, w.conn, w.fixed)
    assert np.array_equal(rp, ro) and np.array_equal(ci, co) and np.array_equal(mp, tm)
    assert ctx.sizes.compact_map == 0


@pytest.mark.parametrize("mesh", ["tiny_tet", "tet_beam", "hex_diff"])
def test_ordering_is_a_permutation(mesh):
    w = synth.make(mesh)
    ctx = _ctx(w)
    perm, snp = ctx.export_ordering()
    assert np.array_equal(np.sort(perm), np.arange(w.n_dofs))
    nfree = int((w.fixed == 0).sum())
    assert np.all(w.fixed[perm[:nfree]] == 0) and np.all(w.fixed[perm[nfree:]] == 1)
    assert snp[0] == 0 and snp[-1] == nfree and np.all(np.diff(snp) > 0)
    assert ctx.sizes.n_levels >= 1
    assert ctx.sizes.factor_lower <= ctx.sizes.factor_entries


@pytest.mark.parametrize("mesh", ["tiny_tet", "tiny_hex", "hex_diff"])
def test_supernodes_cover_the_symbolic_factor(mesh):
    """Panel rows and levels against the structure of the Cholesky factor of
    the permuted free block, found by boolean elimination: every supernode's
    panel holds at least the rows its columns reach, the lower entries sum to
    the reported count, and each column's parent in the elimination tree lies
    in the same supernode or one at a higher level."""
    w = synth.make(mesh)
    ctx = _ctx(w)
    perm, snp = ctx.export_ordering()
    m, lev = ctx.export_supernodes()
    rp, ci, _ = ctx.export_pattern()
    nf = int(snp[-1])
    inv = np.full(w.n_dofs, -1)
    inv[perm[:nf]] = np.arange(nf)
    S = np.zeros((nf, nf), dtype=bool)
    for r in range(w.n_dofs):
        for c in ci[rp[r]:rp[r + 1]]:
            if inv[r] >= 0 and inv[c] >= 0:
                S[inv[r], inv[c]] = S[inv[c], inv[r]] = True
    S = np.tril(S)
    parent = np.full(nf, -1)
    for j in range(nf):
        rows = np.nonzero(S[j + 1:, j])[0] + j + 1
        if rows.size:
            parent[j] = rows[0]
            S[np.ix_(rows, rows)] |= np.tril(np.ones((rows.size, rows.size), dtype=bool))
    sn_of = np.repeat(np.arange(len(m)), np.diff(snp))
    nc = np.diff(snp)
    for s in range(len(m)):
        a, b = snp[s], snp[s + 1]
        reach = np.count_nonzero(S[a:, a:b].any(axis=1))
        assert nc[s] <= reach <= m[s] <= nf - a
    lower = int((m.astype(np.int64) * nc - nc * (nc - 1) // 2).sum())
    assert lower == ctx.sizes.factor_lower
    assert lev.min() == 0 and lev.max() == ctx.sizes.n_levels - 1
    for j in range(nf):
        if parent[j] >= 0 and sn_of[parent[j]] != sn_of[j]:
            assert lev[sn_of[parent[j]]] > lev[sn_of[j]]


@pytest.mark.parametrize("mesh,leaf", [("tiny_tet", 4), ("tiny_hex", 6), ("tet_beam", 0),
                                       ("tet_beam", 8)])
def test_host_factor_applies_inverse(mesh, leaf):
    w = synth.make(mesh)
    q, v = step.rollout(w, w.q0(), w.v0(), 2)[-1]
    s = step.assemble(w, q, v)
    ctx = _ctx(w, leaf=leaf)
    rng = np.random.default_rng(0)
    R = rng.standard_normal((3, w.n_dofs))
    Z = ctx.host_factor_apply(s.vals, R)
    p = s.pat
    for k in range(3):
        ref = solve.dense_cholesky_solve(p.n, p.row_ptr, p.col_idx, s.vals, R[k])
        assert np.abs(Z[k] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_host_factor_rejects_indefinite_matrix():
    w = synth.make("tiny_tet")
    s = step.assemble(w, w.q0(), w.v0())
    ctx = _ctx(w)
    with pytest.raises(_lib.FEError) as ei:
        ctx.host_factor_apply(-s.vals, np.ones((1, w.n_dofs)))
    assert ei.value.code == _lib.FE_EFACTOR


def test_build_pattern_rejects_bad_input():
    w = synth.make("tiny_hex")
    bad = w.conn.copy()
    bad[0, 0] = w.n_nodes + 5
    with pytest.raises(_lib.FEError) as ei:
        FEContext(w.X, bad, w.elem_type, w.fixed, device="cpu")
    assert ei.value.code == _lib.FE_EINVAL
    inv = w.conn.copy()
    inv[0] = inv[0][[1, 0, 3, 2, 5, 4, 7, 6]]    # mirrored hex: negative volume
    with pytest.raises(_lib.FEError) as ei:
        FEContext(w.X, inv, w.elem_type, w.fixed, device="cpu")
    assert ei.value.code == _lib.FE_EINVAL
    with pytest.raises(_lib.FEError):
        FEContext(w.X, w.conn, 6, w.fixed, device="cpu")
    # a free node that belongs to no element (e.g. left behind by a cut)
    X2 = np.vstack([w.X, [[1.0, 1.0, 1.0]]])
    fx2 = np.concatenate([w.fixed, np.zeros(3, np.uint8)])
    with pytest.raises(_lib.FEError) as ei:
        FEContext(X2, w.conn, w.elem_type, fx2, device="cpu")
    assert ei.value.code == _lib.FE_EINVAL and "no element" in str(ei.value)
    fx2[-3:] = 1                                 # fixed: an identity row, accepted
    FEContext(X2, w.conn, w.elem_type, fx2, device="cpu").close()


def test_query_workspace_grows_with_precision():
    w = synth.make("tet_beam")
    ctx = _ctx(w)
    s32 = ctx.query(1)
    s64 = ctx.query(0)
    assert s64.ws_bytes > s32.ws_bytes > 0


def test_bench_refuses_more_than_one_gpu():
    # the benchmark is single-GPU: any --gpus above 1 exits with status 2
    # and a message before any GPU work (so this runs without a GPU)
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for extra in ([], ["--factor-only", "1"], ["--kernel-pass-only"]):
        p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", *extra],
                           stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
        assert p.returncode == 2, (extra, p.stderr[-300:])
        assert "one GPU only" in p.stderr
        assert p.stdout == ""


def test_traffic_record_scaling_and_sweep_families(tmp_path, monkeypatch):
    """The traffic record scales each counter by what it reads for the 1 GiB
    calibration copy, averages a sweep family over all its level launches
    (whatever their tile template arguments) and is honoured only while the
    kernel and tile-schedule sources are unchanged."""
    import csv
    import importlib
    import json
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    bench = importlib.import_module("bench")
    rec_path = tmp_path / "rec.txt"
    monkeypatch.setattr(bench, "_traffic_record", lambda wl: str(rec_path))
    ns = "void fe::(anonymous namespace)::"
    # (kernel, FETCH_SIZE KiB, WRITE_SIZE KiB) per dispatch: the copy reads
    # half its bytes on FETCH_SIZE (scale 2) and all of them on WRITE_SIZE
    disp = [("void at::native::vectorized_elementwise_kernel<4>(int)", 524288.0, 1048576.0),
            (ns + "k_spmv<float, 16>(long, int const*)", 100.0, 10.0),
            (ns + "k_tri_fwd<float, 64, true, 1>(fe::TileDev const*)", 300.0, 6.0),
            (ns + "k_tri_fwd<float, 64, true, 4>(fe::TileDev const*)", 500.0, 2.0),
            (ns + "k_tri_bwd<float, 512, true, 16>(fe::TileDev const*)", 400.0, 4.0)]
    for name, col in (("fetch.csv", 1), ("write.csv", 2)):
        with open(tmp_path / name, "w", newline="") as fh:
            wr = csv.writer(fh)
            wr.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
            for d in disp:
                wr.writerow([d[0], "FETCH_SIZE" if col == 1 else "WRITE_SIZE", d[col]])
    bench._write_traffic_record(str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"),
                                "hex_block", 1024)
    rec = json.load(open(rec_path))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    fwd = rec["kernels"]["k_tri_fwd"]
    assert fwd["dispatches"] == 2
    assert fwd["traffic_bytes_per_launch"] == (400.0 * 2 + 4.0) * 1024
    assert rec["kernels"]["k_spmv<float, 16>"]["traffic_bytes_per_launch"] == (200.0 + 10.0) * 1024
    assert bench._recorded_traffic("hex_block", "k_tri_bwd") == round((800.0 + 4.0) * 1024)
    rec["sources_sha256"][bench.TRAFFIC_SOURCES[1]] = "0" * 64  # a changed tile schedule
    json.dump(rec, open(rec_path, "w"))
    assert bench._recorded_traffic("hex_block", "k_tri_bwd") is None


@pytest.mark.parametrize("mesh", ["hex_diff", "hex_beam"])
@pytest.mark.parametrize("opts", [{}, {"fwd_tile_cols": 64, "fwd_col_groups": 4,
                                       "bwd_tile_rows": 1024, "bwd_tile_cols": 64},
                                  {"fwd_tile_cols": 128, "bwd_tile_rows": 256,
                                   "bwd_tile_cols": 16}])
def test_sweep_tiles_cover_each_lower_panel_entry_once(mesh, opts):
    """The sweeps' tile schedule (per-level extents chosen by the analysis, or
    fixed by the build options) covers every panel entry on or below the
    diagonal of L11^{-1} exactly once in each sweep, with tiles in level order
    (forward ascending, backward descending)."""
    w = synth.make(mesh)
    ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec=1, device="cpu", **opts)
    _, snp = ctx.export_ordering()
    m, lev = ctx.export_supernodes()
    nc = np.diff(snp)
    ext, fwd, bwd = ctx.export_sweep_tiles()
    assert ext.shape == (int(lev.max()) + 1, 4)
    assert set(ext[:, 0]) <= {16, 32, 64, 128} and set(ext[:, 1]) <= {1, 2, 4}
    assert set(ext[:, 2]) <= {256, 512, 1024} and set(ext[:, 3]) <= {16, 32, 64}
    assert all(g == 1 or c == 64 for c, g in ext[:, :2])
    for key, val in opts.items():  # a fixed extent holds on every level it applies to
        col = {"fwd_tile_cols": 0, "fwd_col_groups": 1, "bwd_tile_rows": 2, "bwd_tile_cols": 3}[key]
        assert (ext[:, col] == val).all() or (key == "fwd_col_groups" and
                                              (ext[ext[:, 0] == 64, 1] == val).all())
    for tiles, fwd_dir in ((fwd, True), (bwd, False)):
        tl = lev[tiles[:, 0]]
        assert (np.diff(tl) >= 0).all() if fwd_dir else (np.diff(tl) <= 0).all()
        cover = [np.zeros((int(m[s]), int(nc[s])), dtype=np.int32) for s in range(len(m))]
        for s, r0, c0 in tiles:
            L = lev[s]
            h = 256 if fwd_dir else ext[L, 2]
            wdt = ext[L, 0] * ext[L, 1] if fwd_dir else ext[L, 3]
            cover[s][r0:r0 + h, c0:c0 + wdt] += 1
        for s in range(len(m)):
            low = np.tril(np.ones((int(m[s]), int(nc[s])), dtype=bool))
            assert (cover[s][low] == 1).all(), (mesh, s, fwd_dir)
