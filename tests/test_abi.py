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
    assert lib.nlrmm_strerror(-2) == b"inconsistent or unsupported sizes"
    assert lib.nlrmm_version() >= 100
