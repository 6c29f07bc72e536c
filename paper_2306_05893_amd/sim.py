"""Python front end of the FE step library: torch owns device memory and the
stream; every computation happens in the HIP library behind the C ABI.

``FEContext`` mirrors the C entry points one to one.  ``Simulation`` bundles a
context with the state and parameters of one mesh.  ``RolloutFn`` is the
``torch.autograd.Function`` of a k-step rollout: forward keeps a checkpoint of
(q, v) every ``checkpoint_every`` steps, backward recomputes each segment and
runs the adjoint step (``fe_step_adjoint``) in reverse, returning gradients
with respect to the per-element Young's moduli and the initial state.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class StepOptions:
    rel_tol: float = 1e-8
    max_it: int = 500
    refresh: int = 1
    lag: int = 0
    mode: int = L.FE_FACTOR_DETERMINISTIC
    warm_start: int = 0
    rotate: int = 0

    def c(self):
        return L.fe_step_opts(self.rel_tol, self.max_it, self.refresh, self.lag, self.mode,
                              self.warm_start, self.rotate)


class Params:
    """Physical parameters; E and f_nodal are kept as device tensors."""

    def __init__(self, h, alpha, beta, rho, nu, material, gravity, E, f_nodal=None,
                 device="cuda", mr_c01_share=0.25):
        self.h, self.alpha, self.beta, self.rho, self.nu = h, alpha, beta, rho, nu
        self.material = int(material)
        self.mr_c01_share = float(mr_c01_share)
        self.gravity = [float(g) for g in gravity]
        self.E = torch.as_tensor(np.asarray(E), dtype=torch.float64, device=device).contiguous() \
            if not isinstance(E, torch.Tensor) else E.to(device=device, dtype=torch.float64).contiguous()
        self.f_nodal = None
        if f_nodal is not None:
            f = f_nodal if isinstance(f_nodal, torch.Tensor) else torch.as_tensor(np.asarray(f_nodal))
            self.f_nodal = f.to(device=device, dtype=torch.float64).reshape(-1).contiguous()

    def c(self):
        p = L.fe_params()
        p.h, p.alpha, p.beta, p.rho, p.nu = self.h, self.alpha, self.beta, self.rho, self.nu
        p.material = self.material
        p.pad_ = 0
        for i in range(3):
            p.gravity[i] = self.gravity[i]
        p.E = self.E.data_ptr()
        p.f_nodal = self.f_nodal.data_ptr() if self.f_nodal is not None else None
        p.mr_c01_share = self.mr_c01_share
        return p

    def with_E(self, E):
        q = Params.__new__(Params)
        q.__dict__.update(self.__dict__)
        q.E = E.to(dtype=torch.float64).contiguous()
        return q


@dataclass
class Constraints:
    """k x n_dofs constraint matrix H in CSR form on the device (int32 row
    pointers and columns, FP64 values)."""
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def k(self):
        return int(self.row_ptr.numel()) - 1

    @property
    def nnz(self):
        return int(self.col.numel())

    @staticmethod
    def from_host(H, device="cuda"):
        rp, col, val = H
        return Constraints(torch.as_tensor(np.ascontiguousarray(rp, np.int32), device=device),
                           torch.as_tensor(np.ascontiguousarray(col, np.int32), device=device),
                           torch.as_tensor(np.ascontiguousarray(val, np.float64), device=device))


class FEContext:
    """One library context bound to a caller-owned torch workspace."""

    def __init__(self, X, conn, elem_type, fixed=None, prec=L.FE_PREC_FP64, leaf_nodes=0,
                 n_threads=0, device="cuda", fwd_tile_cols=0, bwd_tile_rows=0,
                 factor_on_gpu=False, factor_max_blocks=0, bwd_tile_cols=0, fwd_col_groups=0):
        self.lib = L.load()
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1)
        conn = np.ascontiguousarray(conn, dtype=np.int32).reshape(-1)
        self.n_nodes = X.size // 3
        self.nen = int(elem_type)
        self.n_elems = conn.size // self.nen
        mesh = L.fe_mesh(self.n_nodes, self.n_elems, int(elem_type),
                         conn.ctypes.data_as(C.c_void_p), X.ctypes.data_as(C.c_void_p))
        fx = None
        if fixed is not None:
            fixed = np.ascontiguousarray(fixed, dtype=np.uint8).reshape(-1)
            fx = fixed.ctypes.data_as(C.c_void_p)
        opts = L.fe_build_opts(int(leaf_nodes), int(fwd_tile_cols), int(bwd_tile_rows),
                               1 if factor_on_gpu else 0, int(n_threads), int(factor_max_blocks),
                               int(bwd_tile_cols), int(fwd_col_groups))
        h = C.c_void_p()
        L.check(self.lib.fe_build_pattern(C.byref(mesh), fx, C.byref(opts), C.byref(h)), None)
        self.h = h
        self.prec = int(prec)
        self.device = torch.device(device)
        self.sizes = self.query(self.prec)
        self.ws = None
        self._mwork = None
        self.bound = False

    # ---- lifetime -------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value is not None:
            if self.bound:
                torch.cuda.synchronize(self.device)
            self.lib.fe_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        return L.check(rc, self.h)

    def _vec(self, t, name, n=None):
        """Validate a device FP64 vector argument before it reaches a kernel."""
        n = self.sizes.n_dofs if n is None else n
        if t is None:
            raise ValueError(f"{name} is None")
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be a contiguous float64 tensor of {n} entries")
        return t

    def _vals(self, A):
        if not isinstance(A, torch.Tensor) or A.device.type != "cuda":
            raise ValueError("A must be a CUDA tensor")
        if A.dtype != self.value_dtype or not A.is_contiguous() or A.numel() != self.sizes.nnz:
            raise ValueError(f"A must be a contiguous {self.value_dtype} tensor of "
                             f"{self.sizes.nnz} entries")
        return A

    def _params(self, p):
        self._vec(p.E, "params.E", self.n_elems)
        if p.f_nodal is not None:
            self._vec(p.f_nodal, "params.f_nodal")
        return p

    # ---- host-only entry points ----------------------------------------
    def query(self, prec):
        s = L.fe_sizes()
        self._chk(self.lib.fe_query(self.h, int(prec), C.byref(s)))
        return s

    def export_pattern(self):
        s = self.sizes
        rp = np.empty(s.n_dofs + 1, dtype=np.int32)
        ci = np.empty(s.nnz, dtype=np.int32)
        mp = np.empty(s.map_len, dtype=np.int32)
        self._chk(self.lib.fe_export_pattern(self.h, rp.ctypes.data_as(C.c_void_p),
                                             ci.ctypes.data_as(C.c_void_p),
                                             mp.ctypes.data_as(C.c_void_p)))
        return rp, ci, mp

    def export_ordering(self):
        s = self.sizes
        perm = np.empty(s.n_dofs, dtype=np.int32)
        snp = np.empty(s.n_supernodes + 1, dtype=np.int32)
        self._chk(self.lib.fe_export_ordering(self.h, perm.ctypes.data_as(C.c_void_p),
                                              snp.ctypes.data_as(C.c_void_p)))
        return perm, snp

    def export_supernodes(self):
        """Rows of each supernode's panel and its assembly-tree level."""
        s = self.sizes
        m = np.empty(s.n_supernodes, dtype=np.int32)
        lev = np.empty(s.n_supernodes, dtype=np.int32)
        self._chk(self.lib.fe_export_supernodes(self.h, m.ctypes.data_as(C.c_void_p),
                                                lev.ctypes.data_as(C.c_void_p)))
        return m, lev

    def export_sweep_tiles(self):
        """The sweeps' tile schedule: per-level extents [n_levels, 4] (forward
        width, forward groups, backward height, backward width) and the
        forward and backward tiles [n, 3] (supernode, r0, c0) in launch order."""
        nl, nf, nb = C.c_int32(), C.c_int32(), C.c_int32()
        self._chk(self.lib.fe_export_sweep_tiles(self.h, C.byref(nl), C.byref(nf), C.byref(nb),
                                                 None, None, None))
        ext = np.empty((nl.value, 4), dtype=np.int32)
        fwd = np.empty((nf.value, 3), dtype=np.int32)
        bwd = np.empty((nb.value, 3), dtype=np.int32)
        self._chk(self.lib.fe_export_sweep_tiles(self.h, None, None, None,
                                                 ext.ctypes.data_as(C.c_void_p),
                                                 fwd.ctypes.data_as(C.c_void_p),
                                                 bwd.ctypes.data_as(C.c_void_p)))
        return ext, fwd, bwd

    def host_factor_apply(self, A_host, r_host):
        """Host-only: factor FP64 CSR values and apply P^{-1} to rows of r."""
        A = np.ascontiguousarray(A_host, dtype=np.float64)
        r = np.ascontiguousarray(np.atleast_2d(r_host), dtype=np.float64)
        z = np.empty_like(r)
        self._chk(self.lib.fe_host_factor_apply(self.h, A.ctypes.data_as(C.c_void_p),
                                                r.ctypes.data_as(C.c_void_p),
                                                z.ctypes.data_as(C.c_void_p), r.shape[0]))
        return z

    # ---- device entry points -------------------------------------------
    @property
    def value_dtype(self):
        return torch.float32 if self.prec == L.FE_PREC_MIXED else torch.float64

    def bind(self):
        if self.bound:
            return
        nbytes = int(self.sizes.ws_bytes)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = self.ws.data_ptr() + off
        self._chk(self.lib.fe_bind(self.h, self.prec, C.c_void_p(self._ws_ptr), nbytes, _stream()))
        self.bound = True

    def new_values(self):
        return torch.zeros(self.sizes.nnz, dtype=self.value_dtype, device=self.device)

    def new_vector(self):
        return torch.zeros(self.sizes.n_dofs, dtype=torch.float64, device=self.device)

    def assemble(self, params: Params, q, v, A=None, b=None):
        self.bind()
        A = self._vals(self.new_values() if A is None else A)
        b = self._vec(self.new_vector() if b is None else b, "b")
        self._vec(q, "q"), self._vec(v, "v"), self._params(params)
        pc = params.c()
        self._chk(self.lib.fe_assemble(self.h, C.byref(pc), _ptr(q), _ptr(v), _ptr(A), _ptr(b),
                                       _stream()))
        return A, b

    def factor_async(self, A, tag):
        self.bind()
        self._vals(A)
        self._chk(self.lib.fe_factor_async(self.h, _ptr(A), int(tag), _stream()))

    def factor_wait(self, tag):
        self._chk(self.lib.fe_factor_wait(self.h, int(tag)))

    def factor_status(self):
        t = C.c_int64()
        rc = self.lib.fe_factor_status(self.h, C.byref(t))
        return rc, t.value

    def factor_install(self):
        t = C.c_int64()
        self._chk(self.lib.fe_factor_install(self.h, C.byref(t), _stream()))
        return t.value

    def factorize_now(self, A, tag=0):
        """Synchronous convenience: factor A and install it."""
        self.factor_async(A, tag)
        self.factor_wait(tag)
        return self.factor_install()

    def pcg_solve(self, A, b, x=None, rel_tol=1e-8, max_it=1000, check=True):
        self.bind()
        x = self._vec(self.new_vector() if x is None else x, "x")
        self._vals(A), self._vec(b, "b")
        st = L.fe_solve_stats()
        rc = self.lib.fe_pcg_solve(self.h, _ptr(A), _ptr(b), _ptr(x), float(rel_tol),
                                   int(max_it), _stream(), C.byref(st))
        if check and rc != L.FE_ENOTCONV:
            self._chk(rc)
        return x, st

    def step(self, q, v, params: Params, opts: StepOptions, a_out=None):
        self.bind()
        self._vec(q, "q"), self._vec(v, "v"), self._params(params)
        if a_out is not None:
            self._vec(a_out, "a_out")
        pc = params.c()
        oc = opts.c()
        st = L.fe_step_stats()
        self._chk(self.lib.fe_step(self.h, _ptr(q), _ptr(v), C.byref(pc), C.byref(oc),
                                   _ptr(a_out), _stream(), C.byref(st)))
        return st

    def step_adjoint(self, q_n, v_n, v_np1, lq_in, lv_in, lq_out, lv_out, dE, params: Params,
                     opts: StepOptions):
        self.bind()
        for t, nm in ((q_n, "q_n"), (v_n, "v_n"), (v_np1, "v_np1"), (lq_in, "lam_q_in"),
                      (lv_in, "lam_v_in"), (lq_out, "lam_q_out"), (lv_out, "lam_v_out")):
            self._vec(t, nm)
        self._vec(dE, "dE", self.n_elems), self._params(params)
        pc = params.c()
        oc = opts.c()
        st = L.fe_solve_stats()
        self._chk(self.lib.fe_step_adjoint(self.h, _ptr(q_n), _ptr(v_n), _ptr(v_np1),
                                           _ptr(lq_in), _ptr(lv_in), _ptr(lq_out), _ptr(lv_out),
                                           _ptr(dE), C.byref(pc), C.byref(oc), _stream(),
                                           C.byref(st)))
        return st

    def spmv(self, A, x, y=None):
        self.bind()
        y = self._vec(self.new_vector() if y is None else y, "y")
        self._vals(A), self._vec(x, "x")
        self._chk(self.lib.fe_spmv(self.h, _ptr(A), _ptr(x), _ptr(y), _stream()))
        return y

    def precond_apply(self, r, A=None, z=None):
        self.bind()
        z = self._vec(self.new_vector() if z is None else z, "z")
        self._vec(r, "r")
        if A is not None:
            self._vals(A)
        self._chk(self.lib.fe_precond_apply(self.h, _ptr(A), _ptr(r), _ptr(z), _stream()))
        return z

    # ---- many right-hand sides and contact (Sec. 6.2)
    def _multi_work(self, k):
        b = C.c_int64()
        self._chk(self.lib.fe_multi_ws_bytes(self.h, int(k), C.byref(b)))
        need = max(int(b.value), 256)
        if self._mwork is None or self._mwork.numel() < need:
            self._mwork = None
            self._mwork = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._mwork

    def _block(self, t, name, k):
        n = self.sizes.n_dofs
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (n, k):
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape ({n}, {k})")
        return t

    def precond_apply_multi(self, R, Z=None):
        """Z = P^{-1} R for the k columns of R (n_dofs x k, DOF-major)."""
        self.bind()
        k = int(R.shape[1]) if R.dim() == 2 else -1
        self._block(R, "R", k)
        Z = self._block(torch.empty_like(R) if Z is None else Z, "Z", k)
        wk = self._multi_work(k)
        self._chk(self.lib.fe_precond_apply_multi(self.h, _ptr(R), _ptr(Z), k, _ptr(wk),
                                                  wk.numel(), _stream()))
        return Z

    def compliance(self, H: "Constraints", want_Z=False, W=None, Z=None):
        """W = H P^{-1} H^T (k x k) with the installed factor; also
        Z = P^{-1} H^T (n_dofs x k) when want_Z."""
        self.bind()
        k = H.k
        W = torch.empty(k, k, dtype=torch.float64, device=self.device) if W is None else W
        if want_Z and Z is None:
            Z = torch.empty(self.sizes.n_dofs, k, dtype=torch.float64, device=self.device)
        if not (W.is_cuda and W.dtype == torch.float64 and W.is_contiguous()
                and W.numel() == k * k):
            raise ValueError("W must be a contiguous float64 CUDA tensor of k x k entries")
        if Z is not None:
            self._block(Z, "Z", k)
        wk = self._multi_work(k)
        self._chk(self.lib.fe_compliance(self.h, k, _ptr(H.row_ptr), _ptr(H.col), _ptr(H.val),
                                         H.nnz, _ptr(W), _ptr(Z), _ptr(wk), wk.numel(),
                                         _stream()))
        return (W, Z) if want_Z else W

    def compliance_noalloc(self, H: "Constraints", W, Z=None):
        """W = H P^{-1} H^T into the caller's W (k x k), and Z = P^{-1} H^T
        into Z (n_dofs x k) when given, through the entry point that
        allocates nothing (its work blocks live in the library's static
        device scratch)."""
        self.bind()
        k = H.k
        if not (W.is_cuda and W.dtype == torch.float64 and W.is_contiguous()
                and W.numel() == k * k):
            raise ValueError("W must be a contiguous float64 CUDA tensor of k x k entries")
        if Z is not None:
            self._block(Z, "Z", k)
        self._chk(self.lib.fe_compliance_noalloc(self.h, k, _ptr(H.row_ptr), _ptr(H.col),
                                                 _ptr(H.val), H.nnz, _ptr(W), _ptr(Z),
                                                 _stream()))
        return W

    def constraint_apply(self, H: "Constraints", x, transpose=False, s_h=1.0, y_in=None,
                         s_y=1.0, y=None):
        """y = s_h op(H) x + s_y y_in with op(H) = H or H^T."""
        self.bind()
        n = self.sizes.n_dofs
        nx, ny = (H.k, n) if transpose else (n, H.k)
        self._vec(x, "x", nx)
        if y_in is not None:
            self._vec(y_in, "y_in", ny)
        y = self._vec(torch.empty(ny, dtype=torch.float64, device=self.device) if y is None
                      else y, "y", ny)
        self._chk(self.lib.fe_constraint_apply(self.h, H.k, _ptr(H.row_ptr), _ptr(H.col),
                                               _ptr(H.val), H.nnz, 1 if transpose else 0,
                                               float(s_h), _ptr(x), float(s_y), _ptr(y_in),
                                               _ptr(y), _stream()))
        return y

    def pgs(self, W, c, lam=None, max_sweeps=100, tol=0.0):
        """Projected Gauss-Seidel on lambda >= 0, W lambda - c >= 0,
        complementary.  Returns (lambda, info) with info = [sweeps, last
        largest change] (device tensors)."""
        self.bind()
        k = int(c.numel())
        self._vec(c, "c", k)
        if not (W.is_cuda and W.dtype == torch.float64 and W.is_contiguous()
                and W.numel() == k * k):
            raise ValueError("W must be a contiguous float64 CUDA tensor of k x k entries")
        lam = torch.zeros(k, dtype=torch.float64, device=self.device) if lam is None else lam
        self._vec(lam, "lam", k)
        info = torch.zeros(2, dtype=torch.float64, device=self.device)
        self._chk(self.lib.fe_pgs(self.h, k, _ptr(W), _ptr(c), _ptr(lam), int(max_sweeps),
                                  float(tol), _ptr(info), _stream()))
        return lam, info

    def contact_solve(self, A, b, H: "Constraints", delta, W=None, sweeps=200, pgs_tol=0.0,
                      rel_tol=1e-8, max_it=1000):
        """The three stages of Sec. 6.2 for A x = b under H x <= delta:
        free motion A x_free = b; lambda from projected Gauss-Seidel on the
        compliance W = H P^{-1} H^T (built from the installed factor when W
        is None) with c = H x_free - delta; motion correction
        x = A^{-1} (b - H^T lambda), started from x_free.
        Returns (x, x_free, lambda, W, stats)."""
        x_free, st_free = self.pcg_solve(A, b, rel_tol=rel_tol, max_it=max_it)
        if W is None:
            W = self.compliance(H)
        c = self.constraint_apply(H, x_free, s_h=1.0, y_in=delta, s_y=-1.0)
        lam, info = self.pgs(W, c, max_sweeps=sweeps, tol=pgs_tol)
        rhs = self.constraint_apply(H, lam, transpose=True, s_h=-1.0, y_in=b, s_y=1.0)
        x, st_corr = self.pcg_solve(A, rhs, x=x_free.clone(), rel_tol=rel_tol, max_it=max_it)
        return x, x_free, lam, W, {"free": st_free, "correction": st_corr, "pgs": info}

    def structure_changed(self, conn, fixed=None):
        """keepStruct test (Sec. 4): True if the element fill sequence
        (device int32 connectivity, element-major) or the fixed DOFs (device
        uint8, None = unchanged) differ from those of this context's map."""
        self.bind()
        if not (conn.is_cuda and conn.dtype == torch.int32 and conn.is_contiguous()):
            raise ValueError("conn must be a contiguous int32 CUDA tensor")
        if conn.numel() % self.nen:
            raise ValueError("conn length is not a multiple of the element's node count")
        if fixed is not None and not (fixed.is_cuda and fixed.dtype == torch.uint8
                                      and fixed.numel() == self.sizes.n_dofs):
            raise ValueError("fixed must be a uint8 CUDA tensor of n_dofs entries")
        ch = C.c_int32()
        self._chk(self.lib.fe_structure_changed(self.h, conn.numel() // self.nen, _ptr(conn),
                                                _ptr(fixed), C.byref(ch), _stream()))
        return bool(ch.value)

    def set_graphs(self, on=True):
        self._chk(self.lib.fe_set_graphs(self.h, 1 if on else 0))

    def set_kernel_timing(self, on=True):
        self._chk(self.lib.fe_set_kernel_timing(self.h, 1 if on else 0))

    def kernel_times(self):
        """Accumulated event times per kernel family since the last call;
        "bytes" holds algorithmic bytes, or flops for the multi_* kinds."""
        ms = (C.c_double * 6)()
        cnt = (C.c_int64 * 6)()
        by = (C.c_double * 6)()
        self._chk(self.lib.fe_kernel_times(self.h, ms, cnt, by, 6))
        names = ["spmv", "trisolve_fwd", "trisolve_bwd", "element", "multi_fwd", "multi_bwd"]
        return {n: {"ms": ms[i], "count": cnt[i], "bytes": by[i]} for i, n in enumerate(names)}

    def reset(self):
        self._chk(self.lib.fe_reset(self.h))


class Simulation:
    """A mesh + parameters + state driven through one FEContext.

    ``workload`` is any object with the attributes of ``synth.Workload``.
    """

    def __init__(self, workload, prec=L.FE_PREC_FP64, device="cuda", leaf_nodes=0, n_threads=0,
                 factor_on_gpu=False, factor_max_blocks=0, bwd_tile_cols=0, fwd_col_groups=0):
        w = workload
        self.w = w
        self.ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, prec, leaf_nodes, n_threads, device,
                             factor_on_gpu=factor_on_gpu, factor_max_blocks=factor_max_blocks)
        self.params = Params(w.h, w.alpha, w.beta, w.rho, w.nu, w.material, w.gravity, w.E,
                             w.f_nodal, device, getattr(w, "mr_c01_share", 0.25))
        self.device = device
        self._build = dict(prec=prec, leaf_nodes=leaf_nodes, n_threads=n_threads,
                           factor_on_gpu=factor_on_gpu, factor_max_blocks=factor_max_blocks)
        self.q = torch.as_tensor(w.X.reshape(-1).copy(), device=device)
        self.v = torch.zeros_like(self.q)

    def set_topology(self, conn, E, fixed=None):
        """Change the element set (e.g. cutting removes elements) keeping
        the nodes and the state (q, v).  The keepStruct test runs on the GPU;
        if the fill sequence is unchanged nothing is rebuilt (fast assembly,
        returns False).  Otherwise the pattern, map, ordering and factor
        structure are rebuilt for the new mesh (full assembly, Sec. 4.2): a
        new context is bound, the old one closed, and the factor schedule
        starts again (returns True).  E: Young's modulus per new element."""
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        dconn = torch.as_tensor(conn.reshape(-1), device=self.device)
        dfx = None if fx is None else torch.as_tensor(fx, device=self.device)
        if not self.ctx.structure_changed(dconn, dfx):
            return False
        import dataclasses
        w = dataclasses.replace(self.w, conn=conn, E=np.asarray(E, dtype=np.float64),
                                fixed=self.w.fixed if fx is None else fx)
        b = self._build
        ctx = FEContext(w.X, w.conn, w.elem_type, w.fixed, b["prec"], b["leaf_nodes"],
                        b["n_threads"], self.device, factor_on_gpu=b["factor_on_gpu"],
                        factor_max_blocks=b["factor_max_blocks"])
        ctx.bind()
        self.ctx.close()
        self.ctx = ctx
        self.w = w
        self.params = self.params.with_E(torch.as_tensor(w.E, device=self.device))
        return True

    def opts(self, **kw):
        base = dict(rel_tol=self.w.rel_tol, max_it=2000, refresh=self.w.refresh, lag=self.w.lag)
        base.update(kw)
        return StepOptions(**base)

    def step(self, opts=None, a_out=None):
        return self.ctx.step(self.q, self.v, self.params, opts or self.opts(), a_out)


class RolloutFn(torch.autograd.Function):
    """q_T = rollout(E, q0, v0) with adjoint gradients (checkpointed)."""

    @staticmethod
    def forward(fctx, E, q0, v0, ctx: FEContext, params: Params, nsteps: int,
                checkpoint_every: int, opts: StepOptions):
        p = params.with_E(E.detach())
        q = q0.detach().clone()
        v = v0.detach().clone()
        ckpt = {0: (q.clone(), v.clone())}
        for n in range(nsteps):
            ctx.step(q, v, p, opts)
            if (n + 1) % checkpoint_every == 0 and n + 1 < nsteps:
                ckpt[n + 1] = (q.clone(), v.clone())
        fctx.ctx, fctx.params, fctx.nsteps, fctx.k, fctx.opts = ctx, p, nsteps, checkpoint_every, opts
        fctx.ckpt = ckpt
        fctx.save_for_backward(E)
        fctx.vT = v.clone()
        return q, v

    @staticmethod
    def backward(fctx, g_q, g_v):
        ctx, p, N, k, opts = fctx.ctx, fctx.params, fctx.nsteps, fctx.k, fctx.opts
        dev = p.E.device
        lq = g_q.detach().to(torch.float64).contiguous().clone() if g_q is not None else \
            torch.zeros(ctx.sizes.n_dofs, dtype=torch.float64, device=dev)
        lv = g_v.detach().to(torch.float64).contiguous().clone() if g_v is not None else \
            torch.zeros_like(lq)
        dE = torch.zeros_like(p.E)
        for s0 in reversed(range(0, N, k)):
            s1 = min(s0 + k, N)
            q, v = (t.clone() for t in fctx.ckpt[s0])
            states = [(q.clone(), v.clone())]
            for _ in range(s0, s1):
                ctx.step(q, v, p, opts)
                states.append((q.clone(), v.clone()))
            for n in reversed(range(s1 - s0)):
                qn, vn = states[n]
                vn1 = states[n + 1][1]
                ctx.step_adjoint(qn, vn, vn1, lq, lv, lq, lv, dE, p, opts)
        return dE, lq, lv, None, None, None, None, None


def rollout(E, q0, v0, ctx, params, nsteps, checkpoint_every=5, opts=None):
    """Differentiable k-step rollout: returns (q_T, v_T)."""
    return RolloutFn.apply(E, q0, v0, ctx, params, nsteps, checkpoint_every,
                           opts or StepOptions())
