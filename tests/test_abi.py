"""CPU checks of the C ABI: the library loads, exports every declared symbol, and rejects
invalid arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2605_06336_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(nlrmm_[a-z0-9_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    names = declared_symbols()
    assert "nlrmm_project" in names and "nlrmm_backproject" in names
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_host_validation_without_device():
    lib = _lib.lib()
    g = _lib.Geom(nx=8, ny=8, x0=-1, y0=-1, d=0.25, nbins=13, s0=-1.42, ds=2.84 / 13)
    b = _lib.Batch(nframes=1, nviews=4, view_off=None)
    # null context / pointers are rejected before any device work
    assert lib.nlrmm_project(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1, 1, None) == -1
    assert lib.nlrmm_backproject(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1, 1, None) == -1
    assert lib.nlrmm_project_dtheta(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1,
                                    None, None, None, None, None, None) == -1
    assert lib.nlrmm_autotune_project(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1, 1,
                                      None) == -1
    assert lib.nlrmm_autotune_backproject(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1, 1,
                                          None) == -1
    assert lib.nlrmm_ctx_set_tune_file(None, b"x") == -1
    c = ctypes.c_int32()
    assert lib.nlrmm_tune_query(None, 0, ctypes.byref(g), ctypes.byref(b), 1,
                                ctypes.byref(c)) == -1
    assert lib.nlrmm_ctx_set_timing(None, 1) == -1
    assert lib.nlrmm_backproject_dtheta(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1, 1,
                                        None) == -1
    assert lib.nlrmm_solver_grid_search(None, ctypes.byref(b), 1, 1, 1, 3, 10, None, None,
                                        None) == -1
    assert lib.nlrmm_solver_offset_sensitivity(None, ctypes.byref(b), 1, 1, 10, 1, None,
                                               None) == -1
    for name in ("nlrmm_fan_project", "nlrmm_fan_backproject", "nlrmm_fan_project_dtheta",
                 "nlrmm_fan_backproject_dtheta"):
        fn = getattr(lib, name)
        assert fn(None, ctypes.byref(g), ctypes.byref(b), 1, 1, 1, 4.0, 1, None) == -1
        # the geometry is checked first, then pointers, the source distance and the batch
        g0 = _lib.Geom(nx=0, ny=8, x0=-1, y0=-1, d=0.25, nbins=13, s0=-1.42, ds=0.2)
        assert fn(None, ctypes.byref(g0), ctypes.byref(b), 1, 1, 1, 4.0, 1, None) == -2
    # the photoacoustic family: null context or geometry
    pg = _lib.PatGeom(n_sensors=4, n_radii=5, n_samples=64, sensor_radius=1.5, radius_step=0.4)
    for name in ("nlrmm_pat_project", "nlrmm_pat_project_dp", "nlrmm_pat_backproject"):
        fn = getattr(lib, name)
        assert fn(None, ctypes.byref(g), ctypes.byref(pg), 1, 1, 0.1, 1, None) == -1
        assert fn(None, ctypes.byref(g), None, 1, 1, 0.1, 1, None) == -1
    # the optical-flow family: null context, then a temporal mode it does not know
    assert lib.nlrmm_of_estimate(None, ctypes.byref(g), 3, 1, 0.05, 1e-3, 10, 1, None) == -1
    assert lib.nlrmm_theta_apply(None, ctypes.byref(g), 3, 2, 1, 1, 1, None) == -1
    assert lib.nlrmm_theta_weights(None, ctypes.byref(g), 3, 2, 1, 1, 1e-3, 1, None) == -1
    assert lib.nlrmm_theta_grad_add(None, ctypes.byref(g), 3, 2, 1, 1, None, 1e-3, 1, 1,
                                    None) == -1
    assert lib.nlrmm_gram_theta(None, ctypes.byref(g), 3, 2, 1, 4, 1, 1, 1, 4, 0, None) == -1
    assert lib.nlrmm_strerror(-2) == b"inconsistent or unsupported sizes"
    assert lib.nlrmm_version() >= 100


def _geom(n, nb, span=2.84):
    return _lib.Geom(nx=n, ny=n, x0=-1.0, y0=-1.0, d=2.0 / n, nbins=nb, s0=-span / 2,
                     ds=span / nb)


def _bwd_limit_ok(g):
    """The backward family's documented limit, restated from the header's comment."""
    import math
    e = math.ceil(g.d * math.sqrt(2.0) / g.ds - 1e-12)
    w = math.ceil(15 * g.d * math.sqrt(2.0) / g.ds) + e + 4
    return 1 <= e <= 4 and w <= 64


def test_geometry_limits_are_checked_on_the_host():
    lib = _lib.lib()
    FWD, BWD = 1, 2
    # the workloads' shapes pass both families
    for n, nb in [(64, 91), (256, 363), (512, 725), (2048, 2897)]:
        g = _geom(n, nb)
        assert lib.nlrmm_check_geom(FWD | BWD, ctypes.byref(g)) == 0, (n, nb)
    # forward family: lines of at most 4096 pixels
    assert lib.nlrmm_check_geom(FWD, ctypes.byref(_geom(4096, 8))) == 0
    assert lib.nlrmm_check_geom(FWD, ctypes.byref(_geom(4097, 8))) == -2
    # backward family: bins no narrower than about 0.38 pixel widths (64^2 with 363 bins fails)
    g = _geom(64, 363)
    assert not _bwd_limit_ok(g)
    assert lib.nlrmm_check_geom(BWD, ctypes.byref(g)) == -2
    assert lib.nlrmm_check_geom(FWD, ctypes.byref(g)) == 0
    # the boundary agrees with the header's formula on a sweep of bin widths
    for nb in range(60, 260, 3):
        g = _geom(64, nb)
        want = 0 if _bwd_limit_ok(g) else -2
        assert lib.nlrmm_check_geom(BWD, ctypes.byref(g)) == want, nb
    # general limits and bad arguments
    assert lib.nlrmm_check_geom(FWD, ctypes.byref(_geom(16385, 8))) == -2
    assert lib.nlrmm_check_geom(FWD, None) == -1
    assert lib.nlrmm_check_geom(4, ctypes.byref(_geom(64, 91))) == -1


def test_entry_points_reject_out_of_range_shapes_before_any_device_work():
    """A geometry beyond an operator family's limits returns NLRMM_ESHAPE from the entry
    point itself, before the context or any pointer is used (here: no context, no device)."""
    lib = _lib.lib()
    b = _lib.Batch(nframes=1, nviews=4, view_off=None)
    big = _geom(4097, 8)        # beyond the forward family
    narrow = _geom(64, 363)     # beyond the backward family
    gb, bb = ctypes.byref(big), ctypes.byref(b)
    gn = ctypes.byref(narrow)
    assert lib.nlrmm_project(None, gb, bb, 1, 1, 1, 1, None) == -2
    assert lib.nlrmm_project_dtheta(None, gb, bb, 1, 1, 1, 1, None, None, None, None,
                                    None) == -2
    assert lib.nlrmm_project_residual(None, gb, bb, 1, 1, 1, 1, None, None) == -2
    assert lib.nlrmm_autotune_project(None, gb, bb, 1, 1, 1, 1, None) == -2
    assert lib.nlrmm_backproject(None, gn, bb, 1, 1, 1, 1, None) == -2
    assert lib.nlrmm_backproject_acc(None, gn, bb, 1, 1, 1, 1, 0, None) == -2
    assert lib.nlrmm_backproject_dtheta(None, gn, bb, 1, 1, 1, 1, None) == -2
    assert lib.nlrmm_autotune_backproject(None, gn, bb, 1, 1, 1, 1, None) == -2
    # the forward family accepts the narrow-bin geometry: only the pointers fail there
    assert lib.nlrmm_project(None, gn, bb, 1, 1, 1, 1, None) == -1
