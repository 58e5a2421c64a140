"""Host logic of the snapshot files (checkpoint / resume), on the CPU with a
stand-in for the solver that keeps the state in a numpy array: the npz layout
(the paper's field names, the time, the grid), the round trip, and the
refusal of a snapshot whose grid differs from the solver's."""
import numpy as np
import pytest

from paper_1908_08557_amd import snapshot


class HostSolver:
    """The parts of cmhd.Solver that snapshot.save/load use, on host arrays."""

    def __init__(self, nx, ny, nz, zbc="solar"):
        self.grid = dict(nx=nx, ny=ny, nz=nz, Lx=8.0, Ly=8.0, z0=0.0, z1=5.0, zbc=zbc)
        self.precision = "fp64"

    def new_state(self):
        g = self.grid
        return np.zeros((8, g["nz"] + 6, g["ny"], g["nx"]))

    def get_fields(self, state, mask, with_ghosts=False):
        assert mask == 0xFF and with_ghosts
        return state.copy()

    def set_fields(self, state, src, mask, with_ghosts=False):
        assert mask == 0xFF and with_ghosts
        state[...] = src
        return state


def test_round_trip_and_layout(tmp_path):
    s = HostSolver(16, 8, 5)
    x = np.random.default_rng(3).standard_normal(s.new_state().shape)
    path = tmp_path / "var.npz"
    snapshot.save(path, s, x, 1.25)
    with np.load(path, allow_pickle=False) as d:
        assert set(snapshot.NAMES) <= set(d.files)
        assert d["lnTT"].shape == (11, 8, 16)
        assert np.array_equal(d["ux"], x[3])
        assert float(d["time"]) == 1.25 and int(d["nz"]) == 5 and str(d["zbc"]) == "solar"
    y, t = snapshot.load(path, s)
    assert t == 1.25 and np.array_equal(y, x)
    z = s.new_state()
    y2, _ = snapshot.load(path, s, z)
    assert y2 is z and np.array_equal(z, x)


@pytest.mark.parametrize("other", [dict(nz=6), dict(nx=32), dict(zbc="periodic")])
def test_grid_mismatch_is_refused(tmp_path, other):
    s = HostSolver(16, 8, 5)
    path = tmp_path / "var.npz"
    snapshot.save(path, s, s.new_state(), 0.0)
    g = dict(s.grid)
    g.update(other)
    t = HostSolver(g["nx"], g["ny"], g["nz"], g["zbc"])
    with pytest.raises(ValueError):
        snapshot.load(path, t)
