"""Shared helpers of the GPU parity tests: run the oracle and the library on
the same seeded workload and compare field by field."""
import copy

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


# the physical field each stored component belongs to (A and u as vectors)
GROUPS = {0: (0, 1, 2), 1: (0, 1, 2), 2: (0, 1, 2), 3: (3, 4, 5), 4: (3, 4, 5), 5: (3, 4, 5),
          6: (6,), 7: (7,)}
# components whose own maximum is no error scale: A_z of a potential-field
# state is a cancellation residue (its tendency is d_z div_h A_h of a field
# whose horizontal divergence nearly vanishes), so it is measured against |A|
RESIDUES = ("Az",)


def _values(arr, f, solar):
    a = arr[f, NG:-NG].ravel()
    if solar and f in (3, 4):
        a = np.concatenate([arr[f, :NG].ravel(), a])   # u_x, u_y lower ghost rows are state
    return a


def field_errors_both(got, ref, solar):
    """Per stored component: max |got - ref| over the interior (plus the
    u_x, u_y lower ghost rows in solar mode) divided (own) by the max norm
    of that component in the oracle result and (group) by the max norm of
    its physical field (A, u, ln rho or ln T)."""
    own, grp = {}, {}
    for f in range(8):
        diff = np.max(np.abs(_values(got, f, solar) - _values(ref, f, solar)))
        s_own = np.max(np.abs(_values(ref, f, solar)))
        s_grp = max(np.max(np.abs(_values(ref, g, solar))) for g in GROUPS[f])
        own[NAMES[f]] = diff / s_own if s_own > 0 else diff
        grp[NAMES[f]] = diff / s_grp if s_grp > 0 else diff
    return own, grp


def field_errors(got, ref, solar):
    """The error each component is held to: relative to its own maximum,
    except the cancellation residues, which are relative to their field."""
    own, grp = field_errors_both(got, ref, solar)
    return {k: (grp[k] if k in RESIDUES else own[k]) for k in own}


def perturbed(w, seed=0):
    """A shallow copy of the workload whose state values are each moved by
    about one unit in the last place (relative 2^-52, seeded random sign)."""
    w2 = copy.copy(w)
    rng = np.random.default_rng(seed)
    w2.state = w.state * (1.0 + rng.choice([-1.0, 1.0], w.state.shape) * 2.0 ** -52)
    return w2


# a component whose float64 result the float64 input does not determine to
# the stated tolerance is held to this multiple of the oracle's own spread
FLOOR_FACTOR = 4.0


def oracle_floor(w, nsteps, dt, ref, t0=0.0, seed=0):
    """How far the float64 input determines the result: per component, the
    own-max relative change of the oracle's nsteps result when every input
    value moves by one unit in the last place.  Two correct float64
    evaluations that round differently differ by about this much (a
    component that is the small residual of large cancelling terms, such as
    the velocity of a stratified box one step from hydrostatic rest, has a
    floor well above 1e-16)."""
    got = oracle_run(perturbed(w, seed), nsteps, dt, t0)
    own, _ = field_errors_both(got, ref, w.grid["zbc"] == "solar")
    return own


def assert_parity(got, ref, solar, tol, label="", floor=None, field_norm=()):
    """Each component relative to its own maximum, at tol or, where the
    oracle's floor (oracle_floor) exceeds tol / FLOOR_FACTOR, at
    FLOOR_FACTOR times that floor; the cancellation residues and the
    components in field_norm relative to their physical field."""
    own, grp = field_errors_both(got, ref, solar)
    errs, lim = {}, {}
    for k in own:
        by_field = k in RESIDUES or k in field_norm
        errs[k] = grp[k] if by_field else own[k]
        lim[k] = tol if (by_field or floor is None) else max(tol, FLOOR_FACTOR * floor[k])
    bad = {k: (v, lim[k]) for k, v in errs.items() if not (v <= lim[k])}
    print(f"[parity] {label} own: " + " ".join(f"{k}={v:.2e}" for k, v in own.items()), flush=True)
    print(f"[parity] {label} field: " + " ".join(f"{k}={v:.2e}" for k, v in grp.items()), flush=True)
    if floor is not None:
        print(f"[parity] {label} oracle floor: "
              + " ".join(f"{k}={v:.2e}" for k, v in floor.items()), flush=True)
    assert not bad, f"{label}: fields above their limit (error, limit): {bad}"
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
