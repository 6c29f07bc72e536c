"""ctypes binding of ``libfe_mi355x.so`` (the C ABI in include/fe.h).

Argument marshalling only: every step of the method runs inside the library.
The library must have been built (``__graft_entry__.build()`` or
``python -m paper_2306_05893_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe_mi355x.so")

FE_OK = 0
FE_EINVAL = -1
FE_ENOMEM = -2
FE_EINVERTED = -3
FE_EINDEF = -4
FE_ENOTCONV = -5
FE_EFACTOR = -6
FE_EBUSY = -7
FE_EDEVICE = -8
FE_ESTATE = -9
ERROR_NAMES = {FE_EINVAL: "FE_EINVAL", FE_ENOMEM: "FE_ENOMEM", FE_EINVERTED: "FE_EINVERTED",
               FE_EINDEF: "FE_EINDEF", FE_ENOTCONV: "FE_ENOTCONV", FE_EFACTOR: "FE_EFACTOR",
               FE_EBUSY: "FE_EBUSY", FE_EDEVICE: "FE_EDEVICE", FE_ESTATE: "FE_ESTATE"}

FE_TET4 = 4
FE_HEX8 = 8
FE_NEO_HOOKEAN = 0
FE_STVK = 1
FE_COROTATIONAL = 2
FE_MOONEY_RIVLIN = 3
FE_PREC_FP64 = 0
FE_PREC_MIXED = 1
FE_FACTOR_DETERMINISTIC = 0
FE_FACTOR_ASYNC = 1


class fe_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("elem_type", C.c_int32),
                ("conn", C.c_void_p), ("X", C.c_void_p)]


class fe_build_opts(C.Structure):
    _fields_ = [("leaf_nodes", C.c_int32), ("fwd_tile_cols", C.c_int32),
                ("bwd_tile_rows", C.c_int32), ("factor_on_gpu", C.c_int32),
                ("n_threads", C.c_int32), ("factor_max_blocks", C.c_int32),
                ("bwd_tile_cols", C.c_int32), ("fwd_col_groups", C.c_int32)]


class fe_params(C.Structure):
    _fields_ = [("h", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("rho", C.c_double), ("nu", C.c_double), ("material", C.c_int32),
                ("pad_", C.c_int32), ("gravity", C.c_double * 3), ("E", C.c_void_p),
                ("f_nodal", C.c_void_p), ("mr_c01_share", C.c_double)]


class fe_sizes(C.Structure):
    _fields_ = [("n_dofs", C.c_int64), ("nnz", C.c_int64), ("n_elems", C.c_int64),
                ("map_len", C.c_int64), ("n_supernodes", C.c_int64), ("n_levels", C.c_int64),
                ("factor_entries", C.c_int64), ("factor_lower", C.c_int64),
                ("factor_flops", C.c_double), ("ws_bytes", C.c_int64),
                ("compact_map", C.c_int32), ("pad_", C.c_int32)]


class fe_solve_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("rel_res", C.c_double),
                ("factor_tag", C.c_int64)]


class fe_step_opts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_it", C.c_int32), ("refresh", C.c_int32),
                ("lag", C.c_int32), ("mode", C.c_int32), ("warm_start", C.c_int32),
                ("rotate_precond", C.c_int32)]


class fe_step_stats(C.Structure):
    _fields_ = [("solve", fe_solve_stats), ("step", C.c_int64), ("factor_lag", C.c_int64)]


# name -> (restype, argtypes)
_P = C.c_void_p
SIGNATURES = {
    "fe_build_pattern": (C.c_int, [C.POINTER(fe_mesh), _P, C.POINTER(fe_build_opts), C.POINTER(_P)]),
    "fe_query": (C.c_int, [_P, C.c_int32, C.POINTER(fe_sizes)]),
    "fe_bind": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P]),
    "fe_export_pattern": (C.c_int, [_P, _P, _P, _P]),
    "fe_export_ordering": (C.c_int, [_P, _P, _P]),
    "fe_export_supernodes": (C.c_int, [_P, _P, _P]),
    "fe_export_sweep_tiles": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "fe_assemble": (C.c_int, [_P, C.POINTER(fe_params), _P, _P, _P, _P, _P]),
    "fe_factor_async": (C.c_int, [_P, _P, C.c_int64, _P]),
    "fe_factor_status": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "fe_factor_wait": (C.c_int, [_P, C.c_int64]),
    "fe_factor_install": (C.c_int, [_P, C.POINTER(C.c_int64), _P]),
    "fe_pcg_solve": (C.c_int, [_P, _P, _P, _P, C.c_double, C.c_int32, _P,
                               C.POINTER(fe_solve_stats)]),
    "fe_step": (C.c_int, [_P, _P, _P, C.POINTER(fe_params), C.POINTER(fe_step_opts), _P, _P,
                          C.POINTER(fe_step_stats)]),
    "fe_step_adjoint": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, C.POINTER(fe_params),
                                  C.POINTER(fe_step_opts), _P, C.POINTER(fe_solve_stats)]),
    "fe_spmv": (C.c_int, [_P, _P, _P, _P, _P]),
    "fe_precond_apply": (C.c_int, [_P, _P, _P, _P, _P]),
    "fe_host_factor_apply": (C.c_int, [_P, _P, _P, _P, C.c_int32]),
    "fe_multi_ws_bytes": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64)]),
    "fe_precond_apply_multi": (C.c_int, [_P, _P, _P, C.c_int32, _P, C.c_int64, _P]),
    "fe_compliance": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.c_int64, _P, _P, _P, C.c_int64,
                                _P]),
    "fe_compliance_noalloc": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.c_int64, _P, _P, _P]),
    "fe_constraint_apply": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.c_int64, C.c_int32,
                                      C.c_double, _P, C.c_double, _P, _P, _P]),
    "fe_pgs": (C.c_int, [_P, C.c_int32, _P, _P, _P, C.c_int32, C.c_double, _P, _P]),
    "fe_structure_changed": (C.c_int, [_P, C.c_int64, _P, _P, C.POINTER(C.c_int32), _P]),
    "fe_set_graphs": (C.c_int, [_P, C.c_int32]),
    "fe_set_kernel_timing": (C.c_int, [_P, C.c_int32]),
    "fe_kernel_times": (C.c_int, [_P, _P, _P, _P, C.c_int32]),
    "fe_reset": (C.c_int, [_P]),
    "fe_destroy": (C.c_int, [_P]),
    "fe_last_error": (C.c_char_p, [_P]),
}

_lib = None


def load():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2306_05893_amd.build or __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class FEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, ctx=None):
    if code != FE_OK:
        msg = load().fe_last_error(ctx)
        raise FEError(code, msg.decode() if msg else "")
    return code
