"""Seeded synthetic inputs for the implicit FE step (meshes, loads, parameters).

This module generates *inputs only*: node coordinates, element connectivity,
Dirichlet masks, per-element Young's moduli, nodal point loads and the scalar
parameters of a run.  It holds none of the method's arithmetic (no shape
functions, no material law, no mass matrix, no assembly); both the FP64 CPU
oracle and the GPU library consume what it produces.

The paper's own meshes (the "Raptor" tetrahedral meshes of its assembly and
preconditioner experiments, and the Liver/Cloth/Cube scenes of its results
section) are not available, so structured stand-ins are used:

* hexahedral beams / blocks on a regular grid (like the paper's hex "Cube"),
* Kuhn (Freudenthal) tetrahedral blocks, optionally with the interior nodes
  jittered, which gives an unstructured-like tet mesh (like the Raptor meshes).

Conventions
-----------
* Node id of grid point (i, j, k) on an (nx+1, ny+1, nz+1) node grid is
  ``i + (nx+1) * (j + (ny+1) * k)`` (i fastest).
* Cells are visited in the same order (i fastest, then j, then k).
* HEX8 local node order follows VTK: (0,0,0), (1,0,0), (1,1,0), (0,1,0) and
  the same four corners at z = 1.
* TET4 (Kuhn split): 6 tets per cube, one per permutation pi of the three axes,
  permutations in lexicographic order; vertices v0 = cube corner (i,j,k),
  v_{m+1} = v_m + e_{pi(m)}.  Tets of odd permutations are negatively oriented,
  so their vertices 1 and 2 are swapped; every tet is then positively
  oriented (checked against the geometry when the mesh is built).
* Random numbers: ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

NEO_HOOKEAN = 0
ST_VENANT_KIRCHHOFF = 1
COROTATIONAL = 2
MOONEY_RIVLIN = 3
MATERIAL_NAMES = {NEO_HOOKEAN: "neo-hookean", ST_VENANT_KIRCHHOFF: "stvk",
                  COROTATIONAL: "corotational", MOONEY_RIVLIN: "mooney-rivlin"}

TET4 = 4
HEX8 = 8

# VTK corner offsets of a trilinear hexahedron.
HEX_CORNERS = np.array(
    [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


def grid_nodes(nx: int, ny: int, nz: int, spacing: float) -> np.ndarray:
    """Rest coordinates [N, 3] of an (nx+1)(ny+1)(nz+1) node grid, i fastest."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    return X * spacing


def _node_id(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def _cells(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def hex_connectivity(nx: int, ny: int, nz: int) -> np.ndarray:
    """HEX8 connectivity [E, 8] (int32), cells i fastest, VTK corner order."""
    ci, cj, ck = _cells(nx, ny, nz)
    conn = np.empty((ci.size, 8), dtype=np.int64)
    for a, (di, dj, dk) in enumerate(HEX_CORNERS):
        conn[:, a] = _node_id(ci + di, cj + dj, ck + dk, nx, ny)
    return conn.astype(np.int32)


def kuhn_connectivity(nx: int, ny: int, nz: int, X: np.ndarray) -> np.ndarray:
    """TET4 Kuhn connectivity [6E_cube, 4] (int32), positively oriented on X."""
    ci, cj, ck = _cells(nx, ny, nz)
    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        verts = [np.stack([ci, cj, ck], axis=1)]
        for m in range(3):
            verts.append(verts[-1] + unit[perm[m]])
        ids = [_node_id(v[:, 0], v[:, 1], v[:, 2], nx, ny) for v in verts]
        tets.append(np.stack(ids, axis=1))
    # interleave so that the 6 tets of a cube are consecutive
    conn = np.stack(tets, axis=1).reshape(-1, 4)
    # orientation: swap vertices 1 and 2 where the signed volume is negative
    d = X[conn[:, 1:]] - X[conn[:, :1]]
    sign = np.linalg.det(np.transpose(d, (0, 2, 1)))
    neg = sign < 0
    conn[neg, 1], conn[neg, 2] = conn[neg, 2].copy(), conn[neg, 1].copy()
    d = X[conn[:, 1:]] - X[conn[:, :1]]
    if not np.all(np.linalg.det(np.transpose(d, (0, 2, 1))) > 0):
        raise ValueError("inverted or degenerate tetrahedron in Kuhn mesh")
    return conn.astype(np.int32)


def boundary_node_mask(nx, ny, nz):
    """bool [N]: True for nodes on any face of the node grid."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                          indexing="ij")
    b = (i == 0) | (i == nx) | (j == 0) | (j == ny) | (k == 0) | (k == nz)
    return b.ravel()


def jitter_interior(X, nx, ny, nz, spacing, amplitude, seed):
    """Shift interior nodes by U(-amplitude, amplitude) * spacing per coordinate."""
    rng = np.random.default_rng(seed)
    shift = rng.uniform(-amplitude, amplitude, size=X.shape) * spacing
    interior = ~boundary_node_mask(nx, ny, nz)
    Xj = X.copy()
    Xj[interior] += shift[interior]
    return Xj


def fixed_face_dofs(X, axis=2, value=0.0, tol=1e-12):
    """uint8 [3N]: 1 for every DOF of the nodes on the plane X[:, axis] == value."""
    on = np.abs(X[:, axis] - value) <= tol
    return np.repeat(on, 3).astype(np.uint8)


def face_traction_loads(nx, ny, nz, total_force, direction):
    """Nodal loads [N, 3] of a uniform traction on the z = max face.

    The total force is spread evenly over the nx*ny face quads; each quad hands
    a quarter of its share to each of its corners (the consistent weights of a
    bilinear face for a uniform traction on a uniform grid).
    """
    N = (nx + 1) * (ny + 1) * (nz + 1)
    loads = np.zeros((N, 3))
    per_corner = total_force / (nx * ny) / 4.0
    dirv = np.asarray(direction, dtype=np.float64)
    dirv = dirv / np.linalg.norm(dirv)
    for j in range(ny):
        for i in range(nx):
            for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                loads[_node_id(i + di, j + dj, nz, nx, ny)] += per_corner * dirv
    return loads


@dataclass
class Workload:
    """Everything one run of the step needs, as plain arrays and scalars."""
    name: str
    elem_type: int                 # TET4 or HEX8
    X: np.ndarray                  # [N, 3] float64 rest coordinates
    conn: np.ndarray               # [E, nen] int32
    fixed: np.ndarray              # [3N] uint8, 1 = Dirichlet DOF
    E: np.ndarray                  # [E] float64 Young's modulus per element
    nu: float
    rho: float
    material: int
    h: float
    alpha: float                   # Rayleigh mass coefficient
    beta: float                    # Rayleigh stiffness coefficient
    gravity: np.ndarray            # [3] body acceleration
    f_nodal: np.ndarray            # [N, 3] nodal point loads
    steps: int = 1
    rel_tol: float = 1e-8
    refresh: int = 1               # factor refresh period R
    lag: int = 0                   # factor lag d (deterministic mode)
    dims: tuple = (0, 0, 0)        # cells per axis of the structured grid
    spacing: float = 0.01
    mr_c01_share: float = 0.25     # Mooney-Rivlin: share of mu/2 carried by C01
    extra: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return self.X.shape[0]

    @property
    def n_elems(self):
        return self.conn.shape[0]

    @property
    def n_dofs(self):
        return 3 * self.X.shape[0]

    def q0(self):
        return self.X.reshape(-1).copy()

    def v0(self):
        return np.zeros(self.n_dofs)


def hex_beam(nx, ny, nz, spacing=0.01, **kw):
    X = grid_nodes(nx, ny, nz, spacing)
    return X, hex_connectivity(nx, ny, nz)


def tet_block(nx, ny, nz, spacing=0.01, jitter=0.0, seed=0):
    X = grid_nodes(nx, ny, nz, spacing)
    if jitter > 0:
        X = jitter_interior(X, nx, ny, nz, spacing, jitter, seed)
    return X, kuhn_connectivity(nx, ny, nz, X)


GRAVITY = np.array([0.0, -9.81, 0.0])


def _base(name, etype, X, conn, dims, spacing, **kw):
    N = X.shape[0]
    E = conn.shape[0]
    d = dict(name=name, elem_type=etype, X=X, conn=conn,
             fixed=fixed_face_dofs(X, 2, 0.0), E=np.full(E, 5000.0), nu=0.45,
             rho=1000.0, material=NEO_HOOKEAN, h=0.01, alpha=0.1, beta=0.1,
             gravity=GRAVITY.copy(), f_nodal=np.zeros((N, 3)), dims=dims,
             spacing=spacing)
    d.update(kw)
    return Workload(**d)


def lognormal_E(n_elems, median, sigma_ln, seed):
    rng = np.random.default_rng(seed)
    return median * np.exp(sigma_ln * rng.standard_normal(n_elems))


def sphere_inclusion_E(X, conn, dims, spacing, n_spheres, radius_cells, E_matrix,
                       E_incl, seed):
    """Two-material field: E_incl for elements whose centroid lies in a sphere."""
    rng = np.random.default_rng(seed)
    ext = np.asarray(dims, dtype=np.float64) * spacing
    centres = rng.uniform(0.0, 1.0, size=(n_spheres, 3)) * ext
    cen = X[conn].mean(axis=1)
    r = radius_cells * spacing
    inside = np.zeros(conn.shape[0], dtype=bool)
    for c in centres:
        inside |= np.sum((cen - c) ** 2, axis=1) <= r * r
    return np.where(inside, E_incl, E_matrix)


def make(name: str, material: int | None = None) -> Workload:
    """The named synthetic workloads.

    tet_beam      5x5x17-node Kuhn tet beam (1536 TET4, 1275 DOFs), NH, gravity,
                  10 steps, exact LDL^T (refresh 1, lag 0), rel-res 1e-10.
    hex_beam      20x20x80 hex beam (32000 HEX8, 107163 DOFs), StVK or NH,
                  E=3000, nu=0.4, 1 N tip traction (-y) on the z-max face,
                  no gravity, 100 steps, refresh every 10 steps.
    tet_block     40^3-cube jittered Kuhn block (384000 TET4, 206763 DOFs),
                  NH, gravity + N(0, 0.01 N) nodal forces, 20 steps, refresh 10.
    hex_diff      10x10x40 hex beam (4000 HEX8, 14883 DOFs), log-normal E
                  (median 5000, sigma_ln 0.3), NH, gravity, 20 steps; target
                  trajectory from a second E field.
    hex_block     48x48x192 hex block (442368 HEX8, 1390179 DOFs), two-material
                  NH (2000 / 20000 Pa in 64 spheres of radius 4 cells), gravity,
                  50 steps, refresh 20.
    Small variants for tests: ``tiny_tet``, ``tiny_hex``.
    """
    sp = 0.01
    if name == "tet_beam":
        dims = (4, 4, 16)
        X, conn = tet_block(*dims, spacing=sp)
        w = _base(name, TET4, X, conn, dims, sp, steps=10, rel_tol=1e-10,
                  refresh=1, lag=0)
    elif name == "hex_beam":
        dims = (20, 20, 80)
        X, conn = hex_beam(*dims, spacing=sp)
        w = _base(name, HEX8, X, conn, dims, sp, E=np.full(conn.shape[0], 3000.0),
                  nu=0.4, material=ST_VENANT_KIRCHHOFF, gravity=np.zeros(3),
                  f_nodal=face_traction_loads(*dims, 1.0, (0.0, -1.0, 0.0)),
                  steps=100, refresh=10, lag=0)
    elif name == "tet_block":
        dims = (40, 40, 40)
        X, conn = tet_block(*dims, spacing=sp, jitter=0.2, seed=0)
        rng = np.random.default_rng(1)
        f = rng.normal(0.0, 0.01, size=X.shape)
        fixed = fixed_face_dofs(X, 2, 0.0).reshape(-1, 3).astype(bool)
        f[fixed] = 0.0
        w = _base(name, TET4, X, conn, dims, sp, f_nodal=f, steps=20, refresh=10)
    elif name == "hex_diff":
        dims = (10, 10, 40)
        X, conn = hex_beam(*dims, spacing=sp)
        w = _base(name, HEX8, X, conn, dims, sp,
                  E=lognormal_E(conn.shape[0], 5000.0, 0.3, 0), steps=20,
                  rel_tol=1e-12, refresh=1)
        w.extra["E_target"] = lognormal_E(conn.shape[0], 5000.0, 0.3, 1)
        w.extra["checkpoint_every"] = 5
        rng = np.random.default_rng(2)
        w.extra["fd_elements"] = np.sort(rng.choice(conn.shape[0], 20, replace=False))
    elif name == "hex_block":
        dims = (48, 48, 192)
        X, conn = hex_beam(*dims, spacing=sp)
        w = _base(name, HEX8, X, conn, dims, sp,
                  E=sphere_inclusion_E(X, conn, dims, sp, 64, 4, 2000.0, 20000.0, 0),
                  steps=50, refresh=20)
        w.extra["E_target"] = sphere_inclusion_E(X, conn, dims, sp, 64, 4, 2000.0,
                                                 20000.0, 1)
        w.extra["checkpoint_every"] = 5
    elif name == "tiny_tet":
        dims = (2, 2, 3)
        X, conn = tet_block(*dims, spacing=sp, jitter=0.15, seed=3)
        w = _base(name, TET4, X, conn, dims, sp, steps=3, rel_tol=1e-12)
    elif name == "tiny_hex":
        dims = (2, 2, 3)
        X, conn = hex_beam(*dims, spacing=sp)
        w = _base(name, HEX8, X, conn, dims, sp, steps=3, rel_tol=1e-12)
    else:
        raise KeyError(name)
    if material is not None:
        w.material = material
    return w


WORKLOADS = ("tet_beam", "hex_beam", "tet_block", "hex_diff", "hex_block")


def random_state(w: Workload, scale: float, seed: int):
    """A seeded smooth deformed state (q, v) near rest.

    q = X + u(X) with u a random affine map plus one smooth sine mode (both of
    relative size ``scale``) and a small nodal noise, ramped linearly to zero
    at the z = min face; v is a smooth random field of size 0.1 m/s.  Fixed
    DOFs keep q = X, v = 0.
    """
    rng = np.random.default_rng(seed)
    X = w.X
    L = np.ptp(X, axis=0).max()
    G = scale * rng.uniform(-1, 1, size=(3, 3))
    k = rng.uniform(0.5, 1.5, size=3) * 2 * np.pi / L
    amp = scale * L / (2 * np.pi) * rng.uniform(-1, 1, size=3)
    u = X @ G.T + np.sin(X @ k)[:, None] * amp[None, :]
    u += 0.01 * scale * w.spacing * rng.uniform(-1, 1, size=X.shape)
    u *= ((X[:, 2] - X[:, 2].min()) / max(np.ptp(X[:, 2]), 1e-30))[:, None]
    q = (X + u).reshape(-1)
    vel = 0.1 * (np.cos(X @ k)[:, None] * rng.uniform(-1, 1, size=3)[None, :])
    v = vel.reshape(-1)
    fixed = w.fixed.astype(bool)
    q[fixed] = w.q0()[fixed]
    v[fixed] = 0.0
    return q, v


def random_vector(n: int, seed: int):
    return np.random.default_rng(seed).standard_normal(n)


def contact_constraints(w: Workload, k: int, seed: int, kind: str = "mixed"):
    """k unilateral contact constraints H x <= delta on the surface y = min of
    the mesh, as a k x n CSR matrix (row_ptr, col, val), plus delta.

    Stand-in for the paper's contact scenes (a liver falling on rigid planes,
    about 246 constraints per step): each row is either a node against a
    slightly tilted rigid plane (3 entries: the plane normal on the node's
    DOFs) or a rigid point against a surface triangle of three nodes of that
    face (9 entries: random barycentric weights times the normal).  kind
    "plane", "triangle" or "mixed" (alternating).  Plane rows use distinct
    nodes and triangles distinct node triples, so the rows are independent.
    Only free nodes are used.  delta is N(0, 1) per constraint.
    """
    rng = np.random.default_rng(seed)
    X = w.X
    ymin = X[:, 1].min()
    free = ~w.fixed.reshape(-1, 3).any(axis=1)
    face = np.flatnonzero((np.abs(X[:, 1] - ymin) <= 1e-12) & free)
    nrm = np.array([0.15, -1.0, 0.1])
    nrm /= np.linalg.norm(nrm)
    n_plane = k if kind == "plane" else (0 if kind == "triangle" else (k + 1) // 2)
    n_tri = k - n_plane
    if n_plane > face.size or 3 * n_tri > face.size:
        raise ValueError("not enough free surface nodes for the constraints")
    plane_nodes = rng.choice(face, n_plane, replace=False)
    tri_nodes = rng.choice(face, 3 * n_tri, replace=False).reshape(n_tri, 3)
    row_ptr, col, val = [0], [], []
    ip = it = 0
    for a in range(k):
        use_plane = kind == "plane" or (kind == "mixed" and a % 2 == 0)
        if use_plane:
            nodes, wts = plane_nodes[ip:ip + 1], np.ones(1)
            ip += 1
        else:
            nodes, wts = tri_nodes[it], rng.dirichlet(np.ones(3))
            it += 1
        for nd, wt in zip(nodes, wts):
            for c in range(3):
                col.append(3 * int(nd) + c)
                val.append(wt * nrm[c])
        row_ptr.append(len(col))
    H = (np.asarray(row_ptr, np.int32), np.asarray(col, np.int32), np.asarray(val, np.float64))
    return H, rng.standard_normal(k)
