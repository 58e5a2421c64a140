"""Pins of the oracle's complex-step tangent (the reference for the GPU
adjoint) against central finite differences of the real oracle."""
import numpy as np

from oracle import mhd as O
from paper_1908_08557_amd import workloads as W


def _box():
    w = W.small_stratified(nx=16, ny=16, nz=12, Lxy=12.0, z1=12.0, nbip=2, t_ramp=0.0)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    return w, F, drv


def test_complex_step_matches_central_differences():
    w, F, drv = _box()
    dt = O.cfl_dt(F, w.grid, w.params)
    rng = np.random.default_rng(0)
    # perturb u, ln rho, ln T and the driver; relative scale of each field
    dF = np.zeros_like(F)
    for c in range(8):
        s = max(1.0, 1e-3 * np.max(np.abs(F[c])))
        dF[c] = s * rng.standard_normal(F[c].shape)
    duh = rng.standard_normal(w.uh_target.shape)
    nsteps = 2
    base, tang = O.run_complex_step(F, dF, duh, 0.0, dt, nsteps, w.grid, w.params, w.lnrho0_z, drv)
    eps = 1e-6

    def fwd(sgn):
        d2 = dict(uh=drv["uh"] + sgn * eps * duh, ah=drv["ah"])
        out, _ = O.run(F + sgn * eps * dF, 0.0, dt, nsteps, w.grid, w.params, w.lnrho0_z, d2)
        return out

    fd = (fwd(+1) - fwd(-1)) / (2 * eps)
    inner = (slice(None), slice(3, -3), slice(3, -3), slice(3, -3))
    for c in range(8):
        a, b = tang[c][inner[1:]], fd[c][inner[1:]]
        scale = np.max(np.abs(a))
        fd_roundoff = 1e-15 * np.max(np.abs(F[c])) / eps
        assert np.max(np.abs(a - b)) <= 1e-6 * scale + fd_roundoff, c
    # the real part is the unperturbed step
    ref, _ = O.run(F, 0.0, dt, nsteps, w.grid, w.params, w.lnrho0_z, drv)
    assert np.max(np.abs(base - ref)[inner]) <= 1e-12 * np.max(np.abs(ref[inner]))


def test_loss_directional_derivative():
    # radiation and conduction off so that dt is Alfven-limited and the loss
    # responds to the driver measurably within three steps
    w, F, drv = _box()
    w.params.update(rad_lnT=np.zeros(0), rad_lnL=np.zeros(0), kappa0=0.0)
    dt = O.cfl_dt(F, w.grid, w.params)
    rng = np.random.default_rng(1)
    duh = rng.standard_normal(w.uh_target.shape)
    target = 0.5 * O.bz_at_height(F, w.grid, w.params, 2.0)
    _, tang = O.run_complex_step(F, np.zeros_like(F), duh, 0.0, dt, 3, w.grid, w.params,
                                 w.lnrho0_z, drv)
    Fn, _ = O.run(F, 0.0, dt, 3, w.grid, w.params, w.lnrho0_z, drv)
    O.fill_ghosts(Fn, w.grid, w.params, w.lnrho0_z)
    bz = O.bz_at_height(Fn, w.grid, w.params, 2.0)
    dbz = O.bz_at_height(tang, w.grid, w.params, 2.0) - w.params["Bext"][2]
    dL = np.sum((bz - target) * dbz)
    eps = 1e-3
    Ls = []
    for sgn in (+1, -1):
        d2 = dict(uh=drv["uh"] + sgn * eps * duh, ah=drv["ah"])
        Fo, _ = O.run(F, 0.0, dt, 3, w.grid, w.params, w.lnrho0_z, d2)
        Ls.append(O.bz_misfit_loss(Fo, w.grid, w.params, 2.0, target))
    fd = (Ls[0] - Ls[1]) / (2 * eps)
    assert abs(fd - dL) <= 1e-6 * abs(dL)
