"""ctypes declarations of the C ABI in include/ehelm.h.

Loads the in-tree libehelm.so and raises if it is missing: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libehelm.so")

EH_OK, EH_NOT_CONVERGED = 0, 1
EH_ERR_ARG, EH_ERR_HIP, EH_ERR_OOM, EH_ERR_STATE = -1, -2, -3, -4

EXPORTED = [
    "eh_default_opts", "eh_create", "eh_ndof", "eh_apply_operator",
    "eh_apply_preconditioner", "eh_block_cycle", "eh_block_apply",
    "eh_block_dims", "eh_solve", "eh_gradient", "eh_misfit", "eh_set_stream",
    "eh_destroy", "eh_last_error", "eh_timer_enable", "eh_timer_read",
    "eh_block_solve", "eh_apply_Z", "eh_power_Z", "eh_misfit_noalloc",
]

KERNEL_CLASSES = {
    "fine_sweep": 0, "fine_resid": 1, "coarse": 2, "restrict": 3, "prolong": 4,
    "dense": 5, "operator": 6, "distribute": 7, "couple": 8, "krylov": 9,
    "fine_first": 10, "fine_down": 11, "fine_up": 12, "coarse_down": 13, "coarse_up": 14,
}


class EhOpts(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int), ("cycle", ctypes.c_int),
        ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
        ("n_damping", ctypes.c_int), ("damping", ctypes.c_double * 8),
        ("alpha", ctypes.c_double), ("mg_precision", ctypes.c_int),
        ("restart", ctypes.c_int), ("abc_width", ctypes.c_int),
        ("abc_sides", ctypes.c_uint), ("gamma0", ctypes.c_double),
        ("intergrid", ctypes.c_int), ("graphs", ctypes.c_int),
        ("autotune", ctypes.c_int), ("fused", ctypes.c_int), ("ap_variant", ctypes.c_int),
        ("coarse_solver", ctypes.c_int), ("drop_converged", ctypes.c_int),
    ]


class EhInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2411_15897_amd/build.py "
                           "(hipcc --offload-arch=gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.eh_default_opts.argtypes = [P(EhOpts)]
    L.eh_default_opts.restype = None
    L.eh_create.argtypes = [P(vp), i32, P(i64), P(dbl), P(dbl), P(dbl), P(dbl), dbl, P(EhOpts), vp]
    L.eh_create.restype = i32
    L.eh_ndof.argtypes = [vp]
    L.eh_ndof.restype = i64
    L.eh_apply_operator.argtypes = [vp, vp, vp, i32]
    L.eh_apply_operator.restype = i32
    L.eh_apply_preconditioner.argtypes = [vp, vp, vp, i32]
    L.eh_apply_preconditioner.restype = i32
    L.eh_block_cycle.argtypes = [vp, i32, vp, vp, i32]
    L.eh_block_cycle.restype = i32
    L.eh_block_apply.argtypes = [vp, i32, i32, vp, vp, i32]
    L.eh_block_apply.restype = i32
    L.eh_block_dims.argtypes = [vp, i32, i32, P(i64)]
    L.eh_block_dims.restype = i32
    L.eh_solve.argtypes = [vp, vp, vp, i32, dbl, i32, P(EhInfo)]
    L.eh_solve.restype = i32
    L.eh_block_solve.argtypes = [vp, i32, vp, vp, i32, dbl, i32, P(EhInfo)]
    L.eh_block_solve.restype = i32
    L.eh_apply_Z.argtypes = [vp, vp, vp, dbl, i32]
    L.eh_apply_Z.restype = i32
    L.eh_power_Z.argtypes = [vp, vp, i32, dbl, i32, P(dbl)]
    L.eh_power_Z.restype = i32
    L.eh_gradient.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.eh_gradient.restype = i32
    L.eh_misfit.argtypes = [vp, vp, vp, i32, vp, i32, vp, P(dbl)]
    L.eh_misfit.restype = i32
    L.eh_misfit_noalloc.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp]
    L.eh_misfit_noalloc.restype = i32
    L.eh_timer_enable.argtypes = [vp, ctypes.c_uint]
    L.eh_timer_enable.restype = i32
    L.eh_timer_read.argtypes = [vp, i32, P(i64), P(dbl), P(dbl)]
    L.eh_timer_read.restype = i32
    L.eh_set_stream.argtypes = [vp, vp]
    L.eh_set_stream.restype = i32
    L.eh_destroy.argtypes = [vp]
    L.eh_destroy.restype = None
    L.eh_last_error.argtypes = [vp]
    L.eh_last_error.restype = ctypes.c_char_p
    _lib = L
    return L
