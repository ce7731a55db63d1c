"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function declared in include/zi.h, and
reject bad arguments before touching the device.
"""
import ctypes
import os
import re

import pytest

from paper_1811_07717_amd import zi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "zi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(zi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("zi_assemble", "zi_transfer_solve", "zi_leadfield", "zi_system_destroy",
              "zi_status_string", "zi_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(zi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    bound = {n for n, _, _ in zi.SIGNATURES}
    assert bound == set(declared_functions())


def test_status_strings():
    L = zi.lib()
    for code in range(-6, 1):
        assert L.zi_status_string(code).decode()
    assert L.zi_status_string(-99).decode() == "unknown status"


def test_tiles_listed():
    names = zi.tile_names()
    assert len(names) >= 8 and all(n.startswith(("lpr", "ring")) for n in names)
    assert len(set(names)) == len(names)


def test_null_arguments_rejected_without_device():
    L = zi.lib()
    h = ctypes.c_void_p()
    assert L.zi_assemble(None, None, -1, None, ctypes.byref(h)) == zi.ZI_EINVAL
    assert b"null" in L.zi_last_error()
    mesh = zi.ZiMesh(3, 1, 1, None, None, None)
    el = zi.ZiElectrodes(1, 1, None, None, None)
    assert L.zi_assemble(ctypes.byref(mesh), ctypes.byref(el), -1, None,
                         ctypes.byref(h)) == zi.ZI_EINVAL
    mesh = zi.ZiMesh(10, 5, 2, 8, 8, 8)     # bad sigma_ncomp
    el = zi.ZiElectrodes(2, 2, 8, 8, ctypes.cast(8, zi.c_f64p))
    assert L.zi_assemble(ctypes.byref(mesh), ctypes.byref(el), -1, None,
                         ctypes.byref(h)) == zi.ZI_EINVAL
    assert b"sigma_ncomp" in L.zi_last_error()
    mesh = zi.ZiMesh(10, 5, 1, 8, 8, 8)
    assert L.zi_assemble(ctypes.byref(mesh), ctypes.byref(el), 10, None,
                         ctypes.byref(h)) == zi.ZI_EINVAL      # ground out of range
    o = zi.ZiSolveOpts()
    assert L.zi_transfer_solve(None, ctypes.byref(o), None, None, None) == zi.ZI_EINVAL
    assert L.zi_leadfield(None, None, 0, None, None, None, None, 0, None) == zi.ZI_EINVAL
    assert L.zi_point_dipoles(None, 1, None, None, None, None, None) == zi.ZI_EINVAL
    assert L.zi_spmm(None, 2, None, None, -1, None, None) == zi.ZI_EINVAL
    info = zi.ZiInfo()
    assert L.zi_get_info(None, ctypes.byref(info)) == zi.ZI_EINVAL
    L.zi_system_destroy(None)
