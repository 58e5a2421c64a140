"""The granulation driver's host bookkeeping in the library (births by random
sequential addition, deaths, advection of the centres), run on the CPU through
the C ABI and compared with the oracle on the same random pools: integer and
placement work, bit-exact.  No GPU: the bookkeeping is host code and needs no
device workspace."""
import os

import numpy as np
import pytest

from oracle import granulation as G
from paper_1908_08557_amd import workloads as W

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1908_08557_amd", "libcmhd.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _vext(p):
    X, Y = G.pixel_coords(p)
    XX, YY = np.meshgrid(X, Y)
    kx, ky = 2 * np.pi / p["Lx"], 2 * np.pi / p["Ly"]
    return np.stack([1.3 * np.sin(ky * YY + 0.4) + 0.2, 0.8 * np.cos(kx * XX - 0.9) - 0.3])


@pytest.mark.parametrize("nx,ny,Lx,Ly", [(64, 64, 6.4, 6.4), (128, 32, 12.8, 3.7),
                                         (256, 256, 25.0, 25.0)])
def test_population_bit_exact_over_updates(nx, ny, Lx, Ly):
    from paper_1908_08557_amd import cmhd
    p = G.params(nx, ny, Lx, Ly)
    u, xi = W.granulation_randoms(20000, 13)
    lib = cmhd.Granulation(p, workspace=False)
    ref = G.Driver(p)
    ve = _vext(p)
    cur = 0
    for t, v in [(0.0, None), (0.02, ve), (0.2, ve), (0.41, None), (0.77, ve)]:
        b = lib.update(t, u[cur:], xi[2 * cur:], vext=v)
        assert b == ref.update(t, u, xi, vext=v)
        cur += b
        got, exp = lib.granules(), ref.gr.array()
        assert got.shape == exp.shape and len(exp) > 0
        assert np.array_equal(got[:, :3], exp[:, :3])        # centres, birth times
        assert np.allclose(got[:, 3:], exp[:, 3:], rtol=1e-15, atol=0)
    lib.close()


def test_invalid_parameters_and_time_order():
    from paper_1908_08557_amd import cmhd
    p = G.params(64, 64, 6.4, 6.4)
    for bad in (dict(nx=48), dict(r_lane=0.7), dict(vmin_frac=0.9), dict(Lx=1.0)):
        q = dict(p)
        q.update(bad)
        with pytest.raises(cmhd.CmhdError):
            cmhd.Granulation(q, workspace=False)
    lib = cmhd.Granulation(p, workspace=False)
    u, xi = W.granulation_randoms(2000, 1)
    lib.update(0.5, u, xi)
    with pytest.raises(cmhd.CmhdError):
        lib.update(0.4, u, xi)
    lib.close()
