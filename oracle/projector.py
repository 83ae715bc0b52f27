"""ctypes wrapper of the FP64 C projector oracle (test infrastructure only).

Builds ``liboracle_strip.so`` from ``strip_oracle.c`` with gcc and OpenMP.
Operator definition: see the header of ``strip_oracle.c`` (strip-area model of
the Radon transform of Section 6.2 at per-view angles, and its fan-beam form).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "strip_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_strip.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        sig = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, ip,
               ctypes.c_int, dp, dp, dp, ctypes.c_int]
        for name in ("ora_project", "ora_backproject", "ora_dtheta", "ora_dtheta_t"):
            f = getattr(lib, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        fsig = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                ctypes.c_int, ip, ctypes.c_int, dp, dp, dp, ctypes.c_int]
        for name in ("ora_fan_project", "ora_fan_backproject", "ora_fan_dtheta",
                     "ora_fan_dtheta_t"):
            f = getattr(lib, name)
            f.argtypes = fsig
            f.restype = ctypes.c_int
        lib.ora_dense.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, dp, dp, dp]
        lib.ora_dense.restype = ctypes.c_int
        lib.ora_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _geom(N, nb):
    return 2.84 / nb, -1.42


def _vo(view_off, V):
    if view_off is None:
        view_off = np.array([0, V], dtype=np.int64)
    return np.ascontiguousarray(view_off, dtype=np.int64)


def max_threads() -> int:
    return _load().ora_max_threads()


# below this many pixel-views a call runs on one thread (every output element is computed
# within one loop iteration, so the result does not depend on the thread count)
SMALL_WORK = 1 << 21


def _run(name, src, theta, out_shape, N, nb, vo, nthreads):
    ds, s0 = _geom(N, nb)
    if nthreads == 0 and src.shape[0] * theta.shape[0] * N * N < SMALL_WORK:
        nthreads = 1
    out = np.zeros(out_shape)
    ip = vo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    getattr(_load(), name)(N, nb, s0, ds, vo.shape[0] - 1, ip, src.shape[0],
                           _p(src), _p(theta), _p(out), nthreads)
    return out


def project(x, theta, nb, view_off=None, nthreads=0):
    """y = A(theta) x.

    x: [N, N] or [F, N, N] (one image per frame) or [C, F, N, N] (C columns).
    Returns [V, nb] for the first two forms, [C, V, nb] for the last.
    """
    x = np.asarray(x, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V = theta.shape[0]
    vo = _vo(view_off, V)
    F = vo.shape[0] - 1
    N = x.shape[-1]
    xs = np.ascontiguousarray(x.reshape((-1, F, N, N)))
    y = _run("ora_project", xs, theta, (xs.shape[0], V, nb), N, nb, vo, nthreads)
    return y if x.ndim == 4 else y[0]


def backproject(y, theta, N, view_off=None, nthreads=0):
    """x = A(theta)^T y.

    y: [V, nb] or [C, V, nb].  Returns [F, N, N] (or [N, N] when F == 1) for a
    2-D y, [C, F, N, N] for a 3-D y.
    """
    y = np.asarray(y, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V, nb = y.shape[-2], y.shape[-1]
    vo = _vo(view_off, V)
    F = vo.shape[0] - 1
    ys = np.ascontiguousarray(y.reshape((-1, V, nb)))
    x = _run("ora_backproject", ys, theta, (ys.shape[0], F, N, N), N, nb, vo, nthreads)
    if y.ndim == 3:
        return x
    return x[0, 0] if F == 1 else x[0]


def dtheta(x, theta, nb, view_off=None, nthreads=0):
    """D[v, j] = d (A(theta) x)[v, j] / d theta_v.  Same shapes as ``project``."""
    x = np.asarray(x, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V = theta.shape[0]
    vo = _vo(view_off, V)
    F = vo.shape[0] - 1
    N = x.shape[-1]
    xs = np.ascontiguousarray(x.reshape((-1, F, N, N)))
    d = _run("ora_dtheta", xs, theta, (xs.shape[0], V, nb), N, nb, vo, nthreads)
    return d if x.ndim == 4 else d[0]


def dtheta_t(r, theta, N, view_off=None, nthreads=0):
    """x = D(theta)^T r, the transpose of ``dtheta`` (sum over views of the angle-derivative
    weights times r).  Same shapes as ``backproject``."""
    r = np.asarray(r, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V, nb = r.shape[-2], r.shape[-1]
    vo = _vo(view_off, V)
    F = vo.shape[0] - 1
    rs = np.ascontiguousarray(r.reshape((-1, V, nb)))
    x = _run("ora_dtheta_t", rs, theta, (rs.shape[0], F, N, N), N, nb, vo, nthreads)
    if r.ndim == 3:
        return x
    return x[0, 0] if F == 1 else x[0]


def dense(N, nb, theta):
    """Dense A(theta) and dA/dtheta, shape [V*nb, N*N] each (tiny grids only)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V = theta.shape[0]
    A = np.zeros((V * nb, N * N))
    dA = np.zeros((V * nb, N * N))
    ds, s0 = _geom(N, nb)
    _load().ora_dense(N, nb, s0, ds, V, _p(theta), _p(A), _p(dA))
    return A, dA


# ---------------------------------------------------------------------------------------
# fan beam (source at distance R from the rotation centre; see strip_oracle.c)
# ---------------------------------------------------------------------------------------
def _run_fan(name, src, theta, out_shape, N, nb, R, vo, nthreads):
    ds, s0 = _geom(N, nb)
    if nthreads == 0 and src.shape[0] * theta.shape[0] * N * N < SMALL_WORK:
        nthreads = 1
    out = np.zeros(out_shape)
    ip = vo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    getattr(_load(), name)(N, nb, s0, ds, float(R), vo.shape[0] - 1, ip, src.shape[0],
                           _p(src), _p(theta), _p(out), nthreads)
    return out


def _fan_fwd(name, x, theta, nb, R, view_off, nthreads):
    x = np.asarray(x, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    N = x.shape[-1]
    V = theta.shape[0]
    vo = _vo(view_off, V)
    F = vo.shape[0] - 1
    xs = np.ascontiguousarray(x.reshape((-1, F, N, N)))
    y = _run_fan(name, xs, theta, (xs.shape[0], V, nb), N, nb, R, vo, nthreads)
    return y if x.ndim == 4 else y[0]


def _fan_bwd(name, y, theta, N, R, view_off, nthreads):
    y = np.asarray(y, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    V, nb = y.shape[-2], y.shape[-1]
    vo = _vo(view_off, V)
    F = vo.shape[0] - 1
    ys = np.ascontiguousarray(y.reshape((-1, V, nb)))
    x = _run_fan(name, ys, theta, (ys.shape[0], F, N, N), N, nb, R, vo, nthreads)
    if y.ndim == 3:
        return x
    return x[0, 0] if F == 1 else x[0]


def fan_project(x, theta, nb, R, view_off=None, nthreads=0):
    """Fan-beam projection (source distance R), same shapes as ``project``."""
    return _fan_fwd("ora_fan_project", x, theta, nb, R, view_off, nthreads)


def fan_dtheta(x, theta, nb, R, view_off=None, nthreads=0):
    """Angle derivative of the fan-beam projection, same shapes as ``dtheta``."""
    return _fan_fwd("ora_fan_dtheta", x, theta, nb, R, view_off, nthreads)


def fan_backproject(y, theta, N, R, view_off=None, nthreads=0):
    """Transpose of ``fan_project``, same shapes as ``backproject``."""
    return _fan_bwd("ora_fan_backproject", y, theta, N, R, view_off, nthreads)


def fan_dtheta_t(r, theta, N, R, view_off=None, nthreads=0):
    """Transpose of ``fan_dtheta``."""
    return _fan_bwd("ora_fan_dtheta_t", r, theta, N, R, view_off, nthreads)
