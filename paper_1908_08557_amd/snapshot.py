"""Snapshots of the state for checkpoint and resume (host npz files).

The field names and the scalar `time` follow the paper's snapshot layout
(Sect. 5.3: datasets lnrho, lnTT, the components of A and u, and the time);
the arrays are [nz+6, ny, nx], z slowest, every plane kept (ghost planes
included, so that the u_x, u_y rows below the photosphere, which are state,
survive a restart).  The grid is stored beside them (sizes, extents, plane
heights, boundary kind).  The data are moved with cmhd_get_fields /
cmhd_set_fields.
"""
from __future__ import annotations

import numpy as np

NAMES = ("ax", "ay", "az", "ux", "uy", "uz", "lnrho", "lnTT")


def save(path, solver, state, t):
    """Write the state and its time to `path` (npz)."""
    f = solver.get_fields(state, 0xFF, with_ghosts=True)
    g = solver.grid
    z = np.asarray(g["z"], dtype=np.float64) if "z" in g else np.array([], dtype=np.float64)
    np.savez(path, **{n: f[i] for i, n in enumerate(NAMES)}, time=np.float64(t),
             nx=g["nx"], ny=g["ny"], nz=g["nz"], Lx=g["Lx"], Ly=g["Ly"], z0=g["z0"], z1=g["z1"],
             zbc=g["zbc"], z=z, precision=solver.precision)


def load(path, solver, state=None):
    """Read a snapshot written by save() into `state` (a new device state if
    None); returns (state, time).  The grid must match the solver's."""
    with np.load(path, allow_pickle=False) as d:
        g = solver.grid
        for key in ("nx", "ny", "nz"):
            if int(d[key]) != g[key]:
                raise ValueError(f"snapshot {key} = {int(d[key])}, solver has {g[key]}")
        if str(d["zbc"]) != g["zbc"]:
            raise ValueError("snapshot boundary kind differs from the solver's")
        f = np.stack([d[n] for n in NAMES])
        t = float(d["time"])
    if state is None:
        state = solver.new_state()
    solver.set_fields(state, f, 0xFF, with_ghosts=True)
    return state, t
