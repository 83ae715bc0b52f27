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

# name -> argtypes (all return int except where noted)
SIGNATURES = {
    "nlrmm_version": [],
    "nlrmm_ctx_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int],
    "nlrmm_project": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_backproject": [_P, _GP, _BP, _I32, _P, _P, _P, _P],
    "nlrmm_project_dtheta": [_P, _GP, _BP, _I32, _P, _P, _P, _P, _P, _P, _P, _P],
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
        _lib = l
    return _lib


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = lib().nlrmm_strerror(rc).decode()
        raise NlrmmError(f"{what} failed: {msg} ({rc})")
