"""Shared helpers of the GPU parity tests: run the oracle and the library on
the same seeded workload and compare field by field."""
import numpy as np

from oracle import mhd as O

NG = 3
NAMES = ("Ax", "Ay", "Az", "ux", "uy", "uz", "lnrho", "lnT")


def oracle_run(w, nsteps, dt, t0=0.0):
    """nsteps oracle steps from the workload's state; returns the compact
    layout [8, nz+6, ny, nx] (interior + the u_h ghost rows are meaningful)."""
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    drv = None
    if w.grid["zbc"] == "solar":
        drv = dict(uh=w.uh_target, ah=w.ah_target)
    F, _ = O.run(F, t0, dt, nsteps, w.grid, w.params, w.lnrho0_z, drv)
    return O.to_compact(F)


def oracle_dt(w):
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    return O.cfl_dt(F, w.grid, w.params)


# the physical field each stored component belongs to: A and u are compared
# as vectors (a component can be a cancellation residue, e.g. A_z driven by
# d_z div_h A_h of a potential field, whose own maximum is no error scale)
GROUPS = {0: (0, 1, 2), 1: (0, 1, 2), 2: (0, 1, 2), 3: (3, 4, 5), 4: (3, 4, 5), 5: (3, 4, 5),
          6: (6,), 7: (7,)}


def _values(arr, f, solar):
    a = arr[f, NG:-NG].ravel()
    if solar and f in (3, 4):
        a = np.concatenate([arr[f, :NG].ravel(), a])   # u_x, u_y lower ghost rows are state
    return a


def field_errors(got, ref, solar):
    """Per stored component: max |got - ref| over the interior (plus the
    u_x, u_y lower ghost rows in solar mode), divided by the max norm of the
    physical field (A, u, ln rho or ln T) in the oracle result."""
    errs = {}
    for f in range(8):
        scale = max(np.max(np.abs(_values(ref, g, solar))) for g in GROUPS[f])
        diff = np.max(np.abs(_values(got, f, solar) - _values(ref, f, solar)))
        errs[NAMES[f]] = diff / scale if scale > 0 else diff
    return errs


def assert_parity(got, ref, solar, tol, label=""):
    errs = field_errors(got, ref, solar)
    bad = {k: v for k, v in errs.items() if not (v <= tol)}
    print(f"[parity] {label} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert not bad, f"{label}: fields above {tol}: {bad}"
    return errs


def oracle_patch_centre(w, k, j, i, dt, h):
    """The oracle's value of zone (k, j, i) after one step, from a
    (2h+1)^3 patch of the initial state around it with periodic wrap at the
    patch edges.  One RK3 step reaches 9 zones (three substages of 3-zone
    stencils), so for h >= 9 + 3 and a zone at least h planes away from the
    z boundaries and below the swamp layer the wrap does not reach the
    centre and the value equals that of the whole-box step."""
    g, p = w.grid, w.params
    n = 2 * h + 1
    ys = np.arange(j - h, j + h + 1) % g["ny"]
    xs = np.arange(i - h, i + h + 1) % g["nx"]
    kz = np.arange(k - h, k + h + 1) + NG
    patch = w.state[:, kz][:, :, ys][:, :, :, xs]
    dx, dy = g["Lx"] / g["nx"], g["Ly"] / g["ny"]
    zall = O.zk(g)
    grid = dict(nx=n, ny=n, nz=n, Lx=n * dx, Ly=n * dy, zbc="periodic")
    if "z" in g:
        # heights of the patch planes and of the planes its stencils reach
        grid.update(z=zall[k - h:k + h + 1 + 2 * NG], z0=zall[k - h + NG], z1=zall[k + h + NG])
    else:
        dz = O.spacings(g)[2]
        grid.update(z0=zall[k - h + NG], z1=zall[k - h + NG] + n * dz)
    state = np.zeros((8, n + 2 * NG, n, n))
    state[:, NG:NG + n] = patch
    F = O.from_compact(state)
    O.fill_ghosts(F, grid, p, None)
    F = O.rk3_step(F, 0.0, dt, grid, p, None, None)
    return F[:, NG + h, NG + h, NG + h]
