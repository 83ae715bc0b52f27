"""ctypes binding of libnlrmm.so (the C ABI in include/nlrmm.h).

Argument marshalling only: every computation runs in the library's HIP kernels.
There is no fallback: importing a function whose library is missing raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlrmm.so")


class NlrmmError(RuntimeError):
    pass


class Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("d", ctypes.c_double),
                ("nbins", ctypes.c_int32), ("s0", ctypes.c_double), ("ds", ctypes.c_double)]


class Batch(ctypes.Structure):
    _fields_ = [("nframes", ctypes.c_int32), ("nviews", ctypes.c_int64),
                ("view_off", ctypes.c_void_p)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_GP = ctypes.POINTER(Geom)
_BP = ctypes.POINTER(Batch)


class PatGeom(ctypes.Structure):
    _fields_ = [("n_sensors", ctypes.c_int32), ("n_radii", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("sensor_radius", ctypes.c_double),
                ("radius_step", ctypes.c_double)]


class SolverCfg(ctypes.Structure):
    _fields_ = [("kmin", ctypes.c_int32), ("kmax", ctypes.c_int32), ("solves", ctypes.c_int32),
                ("eps", ctypes.c_double), ("tau", ctypes.c_double), ("lam_fix", ctypes.c_double),
                ("param_update", ctypes.c_int32), ("param_mode", ctypes.c_int32),
                ("maxiter_p", ctypes.c_int32), ("mu_rel", ctypes.c_double),
                ("c1", ctypes.c_double), ("beta", ctypes.c_double), ("alpha0", ctypes.c_double),
                ("armijo_trials", ctypes.c_int32), ("breakdown_tol", ctypes.c_double),
                ("temporal", ctypes.c_int32), ("gram_precision", ctypes.c_int32),
                ("compress_precision", ctypes.c_int32), ("lam_hi", ctypes.c_double),
                ("sens_iters", ctypes.c_int32), ("of_iters", ctypes.c_int32),
                ("of_gamma", ctypes.c_double), ("of_ridge", ctypes.c_double),
                ("of_every", ctypes.c_int32)]

# name -> argtypes (all return int except where noted)
SIGNATURES = {
    "nlrmm_version": [],
    "nlrmm_check_geom": [_I32, _GP],
    "nlrmm_ctx_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int],
    "nlrmm_ctx_set_timing": [_P, _I32],
    "nlrmm_autotune_project": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_autotune_backproject": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_ctx_set_tune_file": [_P, ctypes.c_char_p],
    "nlrmm_tune_query": [_P, _I32, _GP, _BP, _I32, ctypes.POINTER(ctypes.c_int32)],
    "nlrmm_ctx_kernel_ms": [_P, _I32, ctypes.POINTER(ctypes.c_float)],
    "nlrmm_ctx_kernel_avg": [_P, _I32, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_int32)],
    "nlrmm_project": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_backproject": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_backproject_dtheta": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_project_dtheta": [_P, _GP, _BP, _I32, _P, _P, _P, _P, _P, _P, _P, _P],
    "nlrmm_backproject_acc": [_P, _GP, _BP, _I32, _P, _P, _P, _I32, _P],
    "nlrmm_backproject_noalloc": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_of_estimate": [_P, _GP, _I32, _P, ctypes.c_double, ctypes.c_double, _I32, _P, _P],
    "nlrmm_theta_apply": [_P, _GP, _I32, _I32, _P, _P, _P, _P],
    "nlrmm_theta_weights": [_P, _GP, _I32, _I32, _P, _P, ctypes.c_double, _P, _P],
    "nlrmm_theta_grad_add": [_P, _GP, _I32, _I32, _P, _P, _P, ctypes.c_double, _P, _P, _P],
    "nlrmm_gram_theta": [_P, _GP, _I32, _I32, _P, _I32, _P, _P, _P, _I32, _I32, _P],
    "nlrmm_pat_project": [_P, _GP, ctypes.POINTER(PatGeom), _I32, _P, ctypes.c_double, _P, _P],
    "nlrmm_pat_project_dp": [_P, _GP, ctypes.POINTER(PatGeom), _I32, _P, ctypes.c_double, _P,
                             _P],
    "nlrmm_pat_backproject": [_P, _GP, ctypes.POINTER(PatGeom), _I32, _P, ctypes.c_double, _P,
                              _P],
    "nlrmm_fan_project": [_P, _GP, _BP, _I32, _P, _P, ctypes.c_double, _P, _P],
    "nlrmm_fan_backproject": [_P, _GP, _BP, _I32, _P, _P, ctypes.c_double, _P, _P],
    "nlrmm_fan_project_dtheta": [_P, _GP, _BP, _I32, _P, _P, ctypes.c_double, _P, _P],
    "nlrmm_fan_backproject_dtheta": [_P, _GP, _BP, _I32, _P, _P, ctypes.c_double, _P, _P],
    "nlrmm_project_residual": [_P, _GP, _BP, _P, _P, _P, _P, _P, _P],
    "nlrmm_tv_weights": [_P, _GP, _I32, _I32, _P, _D, _P, _P],
    "nlrmm_gram_psi": [_P, _GP, _I32, _I32, _I32, _P, _P, _P, _I32, _I32, _P],
    "nlrmm_gks_solve": [_P, _I32, _P, _P, _I32, _P, _P, _D, _P, _P, _P, _P],
    "nlrmm_gks_expand": [_P, _GP, _BP, _P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _P,
                         _D, _P, _P],
    "nlrmm_recycle_compress": [_P, _I64, _I64, _I32, _I32, _P, _P, _P, _P, _I32, _P, _P, _P,
                               _I32, _P, _P],
    "nlrmm_solver_create": [_P, _GP, _I32, _I64, ctypes.POINTER(SolverCfg),
                            ctypes.POINTER(ctypes.c_void_p)],
    "nlrmm_solver_init": [_P, _BP, _P, _P, _P],
    "nlrmm_solver_outer": [_P, _BP, _P, _P, _D, _P],
    "nlrmm_solver_grid_search": [_P, _BP, _P, _P, _P, _I32, _I32, _P, _P, _P],
    "nlrmm_solver_offset_sensitivity": [_P, _BP, _P, _P, _I32, _P, _P, _P],
    "nlrmm_solver_state": [_P, _P, _P, _P, _P, _P],
    "nlrmm_solver_read": [_P, _P, _P, _P, _P],
    "nlrmm_solver_set_launch": [_P, _I32, _P, _I32],
}


def lib():
    """Load libnlrmm.so (raises NlrmmError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NlrmmError(f"{LIB_PATH} not found: build it with "
                             "`python -m paper_2605_06336_amd.build` (hipcc, gfx950)")
        l = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        l.nlrmm_strerror.argtypes = [ctypes.c_int]
        l.nlrmm_strerror.restype = ctypes.c_char_p
        l.nlrmm_ctx_destroy.argtypes = [ctypes.c_void_p]
        l.nlrmm_ctx_destroy.restype = None
        l.nlrmm_solver_destroy.argtypes = [ctypes.c_void_p]
        l.nlrmm_solver_destroy.restype = None
        _lib = l
    return _lib


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = lib().nlrmm_strerror(rc).decode()
        raise NlrmmError(f"{what} failed: {msg} ({rc})")
