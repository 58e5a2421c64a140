"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and the binding's structures match the header layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmhd.h")
LIB = os.path.join(ROOT, "paper_1908_08557_amd", "libcmhd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmhd_[a-z0-9_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1908_08557_amd import cmhd
    assert sorted(cmhd.exported_symbols()) == declared_functions()


def test_struct_layout_matches_header():
    from paper_1908_08557_amd import cmhd
    # cmhd_grid: 3 ints, 4 doubles, 2 ints (natural alignment)
    assert ctypes.sizeof(cmhd.CmhdGrid) == 56
    # cmhd_params: 8 + 3 + 1 + 9 doubles, int (padded), 2*16 doubles, 5 doubles
    assert ctypes.sizeof(cmhd.CmhdParams) == (21 * 8) + 8 + 32 * 8 + 5 * 8 + 5 * 8
    assert cmhd.CmhdParams.n_rad.offset == 21 * 8
    # cmhd_gran_params: 2 ints, 11 doubles
    assert ctypes.sizeof(cmhd.CmhdGranParams) == 8 + 11 * 8
    assert cmhd.CmhdGranParams.f_rot.offset == 8 + 10 * 8


def test_params_marshalling_roundtrip():
    from paper_1908_08557_amd import cmhd
    from paper_1908_08557_amd import workloads as W
    w = W.strat64()
    p = cmhd.make_params(w.params)
    assert p.n_rad == len(w.params["rad_lnT"])
    assert p.rad_lnT[3] == w.params["rad_lnT"][3]
    assert p.tau_u == w.params["tau_u"] and p.g_z == -274.0
    g = cmhd.make_grid(w.grid, "fp32_split")
    assert (g.nx, g.ny, g.nz, g.zbc, g.prec) == (64, 64, 64, 1, 1)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_init_rejects_invalid_grids_before_touching_a_device():
    # parameter validation is host logic: every case returns CMHD_EINVAL on
    # the CPU (a valid one would go on to look for a gfx950 device)
    import numpy as np

    from paper_1908_08557_amd import cmhd
    from paper_1908_08557_amd import workloads as W
    lib = cmhd.load()
    w = W.small_stratified(32, 32, 12)
    n = 12 + 6
    lr = np.ascontiguousarray(w.lnrho0_z)
    lt = np.ascontiguousarray(w.lnT0_z)
    dp = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def init(grid, params, z=None, lnr=lr, lnt=lt):
        g = cmhd.make_grid(grid)
        p = cmhd.make_params(params)
        out = ctypes.c_void_p()
        zz = None if z is None else np.ascontiguousarray(z, dtype=np.float64)
        return lib.cmhd_init_grid_z(ctypes.byref(g), ctypes.byref(p), dp(zz), dp(lnr), dp(lnt),
                                    None, ctypes.byref(out))

    bad_grids = [dict(nx=24), dict(ny=2048), dict(nz=4), dict(Lx=-1.0), dict(z1=-5.0)]
    for b in bad_grids:
        g = dict(w.grid)
        g.update(b)
        assert init(g, w.params) == cmhd.CMHD_EINVAL, b
    bad_params = [dict(gamma=1.0), dict(eta=-1.0), dict(z_t=0.0, z_s=1.0),
                  dict(nc_tau=1.0, nc_lnrho0_z=None)]
    for b in bad_params:
        p = dict(w.params)
        p.update(b)
        if b.get("nc_tau"):
            assert init(w.grid, p, lnt=None) == cmhd.CMHD_EINVAL, b
        else:
            assert init(w.grid, p) == cmhd.CMHD_EINVAL, b
    # non-uniform heights: not increasing, or with periodic boundaries
    z = np.linspace(0.0, 10.0, n)
    z[7] = z[6]
    assert init(w.grid, w.params, z=z) == cmhd.CMHD_EINVAL
    gp = dict(w.grid)
    gp["zbc"] = "periodic"
    assert init(gp, w.params, z=np.linspace(0.0, 10.0, n)) == cmhd.CMHD_EINVAL
    # solar mode without the ln rho0 profile
    assert init(w.grid, w.params, lnr=None) == cmhd.CMHD_EINVAL
