"""CPU checks of the C-ABI libraries: they load, export every function
include/hk.h declares, and answer the calls that need no device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_11174_amd import build, hk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hk_[a-zA-Z_]+)\s*\(", src)) - {"hk_alloc_fn", "hk_free_fn"})


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_library_exports_every_declared_symbol(prec):
    path = build.lib_path(prec)
    if not os.path.exists(path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(path)
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(hk.ABI_SYMBOLS) <= set(names)


@pytest.mark.parametrize("prec,size", [("f32", 4), ("f64", 8)])
def test_host_only_calls(prec, size):
    if not os.path.exists(build.lib_path(prec)):
        pytest.skip("library not built")
    L = hk.load(prec)
    assert L.hk_real_size() == size
    assert L.hk_strerror(-1) == b"invalid argument"
    assert L.hk_strerror(0) == b"ok"
    # argument validation happens before any device work
    h = ctypes.c_void_p()
    grid = hk.GridDesc(nx=0, ny=8, nz=8, bc_x=1, dx=0.2, dy=0.2, dz=0.2, dt=0.1)
    sps = (hk.SpeciesDesc * 6)()
    las = hk.LaserDesc()
    run = hk.RunDesc()
    assert L.hk_create(ctypes.byref(grid), sps, 0, ctypes.byref(las), ctypes.byref(run),
                       ctypes.byref(h)) == -1
    # a time step above the Courant limit is rejected
    grid.nx = 8
    grid.dt = 0.2
    assert L.hk_create(ctypes.byref(grid), sps, 0, ctypes.byref(las), ctypes.byref(run),
                       ctypes.byref(h)) == -1
    assert L.hk_step(None, 1) == -1


def test_config_marshalling_matches_header_layout():
    # the binding's structs must have the sizes the header implies
    assert ctypes.sizeof(hk.GridDesc) == 4 * 4 + 4 * 8
    assert ctypes.sizeof(hk.SpeciesDesc) == 10 * 4 + 6 * 8 + 8 * 8 + 8        # ... ip_ev[8], gamma_ad
    assert ctypes.sizeof(hk.LaserDesc) == 4 * 4 + 5 * 8
    assert ctypes.sizeof(hk.Diag) == 8 + 8 + 2 * 8 + 4 * 6 * 8 + 8 * 8 + 6 * 8  # ... fluid_th[6]


def test_qed_tables_match_oracle(oracle_mod):
    # the library builds its tables with its own Airy functions (backward ODE
    # integration) and quadrature; the oracle with Bessel integrals and Simpson
    from paper_2510_11174_amd import hk
    We, Wb, Xe, Xb = hk.qed_tables("f32")
    oWe, oWb, oXe, oXb = oracle_mod.qed_tables()
    np.testing.assert_allclose(We, oWe, rtol=1e-10, atol=0)
    live = (oWb > 1e-200) & (Wb > 1e-200)      # rows where the pair rate does not underflow
    np.testing.assert_allclose(Wb[live], oWb[live], rtol=1e-10, atol=0)
    assert np.all(Wb[~live] < 1e-200) and np.all(oWb[~live] < 1e-200)
    np.testing.assert_allclose(Xe, oXe, rtol=0, atol=1e-9)
    np.testing.assert_allclose(Xb[live], oXb[live], rtol=0, atol=1e-7)
    f64 = hk.qed_tables("f64")
    np.testing.assert_array_equal(f64[0], We)
