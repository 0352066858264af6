"""The C-ABI library loads on a machine without a GPU, exports every symbol
its header declares, and rejects invalid parameters before touching the
device."""
import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(ij3?_\w+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    from paper_1702_04487_amd import lbm
    L = lbm.load()
    declared = _declared()
    assert declared, "no declarations found"
    assert declared == set(lbm.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_invalid_parameters_are_rejected_without_a_device():
    from paper_1702_04487_amd import lbm
    L = lbm.load()
    good = W.config_nozzle_small()["params"]
    bad_cases = [dict(good, nx=2), dict(good, tau_ink=0.5), dict(good, rho_amb=2.0),
                 dict(good, width=0.0), dict(good, theta_inner=181.0), dict(good, bc_y=7),
                 dict(good, t_neg=-1), dict(good, nozzle_w=70, nozzle_x0=1, nozzle_len=10),
                 dict(good, nx=60000, ny=60000),
                 dict(good, nx=64, ny=65536),            # rows beyond the 16-bit limit
                 dict(good, nx=2240, ny=65535)]          # 15 * ny * pitch >= 2^31
    for bad in bad_cases:
        p = lbm.to_params(bad)
        h = ctypes.c_void_p()
        assert L.ij_create(ctypes.byref(p), ctypes.byref(h)) == lbm.IJ_ERR_INVALID_ARG
        assert not h.value
        assert L.ij_last_error(None)
        n = ctypes.c_size_t(0)
        assert L.ij_required_bytes(ctypes.byref(p), ctypes.byref(n)) == lbm.IJ_ERR_INVALID_ARG


def test_required_bytes_uses_aligned_pitch():
    from paper_1702_04487_amd import lbm
    L = lbm.load()
    for nx, pitch in [(64, 64), (100, 128), (2048, 2048), (3, 64)]:
        p = lbm.to_params(W.base_params(nx, 40))
        n = ctypes.c_size_t(0)
        assert L.ij_required_bytes(ctypes.byref(p), ctypes.byref(n)) == lbm.IJ_OK
        assert n.value == 40 * pitch * (14 * 4 + 2)


def test_null_handles_are_safe():
    from paper_1702_04487_amd import lbm
    L = lbm.load()
    L.ij_destroy(None)
    assert L.ij_step(None, 1, None) == lbm.IJ_ERR_INVALID_ARG
    assert L.ij_time(None) == -1
    assert L.ij_params_default(None) == lbm.IJ_ERR_INVALID_ARG


def test_batch_rejects_invalid_cases_without_a_device():
    from paper_1702_04487_amd import lbm
    L = lbm.load()
    good = W.config_nozzle_small()["params"]
    for cases in ([good, dict(good, tau_ink=0.4)], [good, dict(good, diag_every=7)]):
        arr = (lbm.IJParams * len(cases))()
        for i, c in enumerate(cases):
            arr[i] = lbm.to_params(c)
        h = ctypes.c_void_p()
        assert L.ij_batch_create(arr, len(cases), ctypes.byref(h)) == lbm.IJ_ERR_INVALID_ARG
        assert not h.value
        assert L.ij_batch_last_error(None)
    h = ctypes.c_void_p()
    assert L.ij_batch_create(None, 0, ctypes.byref(h)) == lbm.IJ_ERR_INVALID_ARG
    L.ij_batch_destroy(None)
    assert L.ij_batch_size(None) == -1 and L.ij_batch_time(None) == -1


def test_largest_lattice_is_accepted():
    from paper_1702_04487_amd import lbm
    L = lbm.load()
    p = lbm.to_params(W.base_params(2048, 65535, bc_y=W.BC_PERIODIC))
    n = ctypes.c_size_t(0)
    assert L.ij_required_bytes(ctypes.byref(p), ctypes.byref(n)) == lbm.IJ_OK
    assert n.value == 65535 * 2048 * (14 * 4 + 2)


def test_3d_invalid_parameters_are_rejected_without_a_device():
    """ij3_create validates parameters and the open-row geometry on the host
    before any device call."""
    import numpy as np
    from paper_1702_04487_amd import lbm, lbm3d
    L = lbm.load()
    c = W.config_round_nozzle_small()
    good = c["params"]
    bad_cases = [dict(good, nz=2), dict(good, nx=2), dict(good, tau_phi=0.5), dict(good, rho_amb=1.5),
                 dict(good, width=-1.0), dict(good, theta_outer=-3.0), dict(good, bc_y=5),
                 dict(good, t_idle=-1), dict(good, nx=70000)]
    for bad in bad_cases:
        p = lbm3d.to_params3(bad)
        h = ctypes.c_void_p()
        assert L.ij3_create(ctypes.byref(p), None, ctypes.byref(h)) == lbm.IJ_ERR_INVALID_ARG, bad
        assert not h.value
        assert L.ij3_last_error(None)
    wall = c["wall"].copy()
    wall[1, 10, 16] = W.WALL_OUTER          # open bottom row: fluid with a wall directly above
    wall[0, 10, 16] = W.FLUID
    h = ctypes.c_void_p()
    p = lbm3d.to_params3(good)
    r = L.ij3_create(ctypes.byref(p), np.ascontiguousarray(wall).ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    assert r == lbm.IJ_ERR_INVALID_ARG and b"open row" in L.ij3_last_error(None)
    wall = c["wall"].copy()
    wall[5, 5, 5] = 7
    r = L.ij3_create(ctypes.byref(p), np.ascontiguousarray(wall).ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    assert r == lbm.IJ_ERR_INVALID_ARG
