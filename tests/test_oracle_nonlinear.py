"""Pins of the oracle's nonlinear right-hand-side terms that single Fourier
modes see only at second order, and of the radiative and nudging limits of
its time step.

Each term is compared with an independent route: the same physical quantity
written in conservative form and differentiated spectrally on a finer
periodic grid (exact for these smooth fields to ~1e-12), so that the oracle's
expanded, non-conservative form must converge to it at sixth order.  A
dropped term, a flipped sign or a wrong factor in the expansion leaves an
O(1) difference that does not converge.

  * continuity, mass diffusion of Sect. 2.5 in ln rho form:
    D_rho (lap ln rho + |grad ln rho|^2) = D_rho lap(rho) / rho
  * compressible viscous force (constant nu; reading):
    nu (lap u + grad div u / 3 + 2 S.grad ln rho) = div(2 rho nu S) / rho
  * Lorentz force per unit mass with non-uniform density:
    J x B / rho with B = curl A + B_ext, mu0 J = curl B
"""
import math

import numpy as np

from oracle import mhd as O
from paper_1908_08557_amd import workloads as W

NG = 3
L = 2 * np.pi


def _spectral_ops(n):
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    k = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    Kv = (KX, KY, KZ)

    def d(f, i):
        return np.real(np.fft.ifftn(1j * Kv[i] * np.fft.fftn(f)))

    return (X, Y, Z), d


def _box(n, lnrho_fun, u_fun=None, A_fun=None, **par):
    """Periodic 2 pi box, ln T = 0, the given ln rho, u and A (functions of
    X, Y, Z on the compact layout's planes, ghosts included)."""
    w = W.periodic_box(n, amp_A=0.0, amp_u=0.0, eta=0.0, nu=0.0)
    w.params.update(par)
    z, _ = W.z_coords(w.grid)
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    w.state[6] = lnrho_fun(X, Y, Z)
    if u_fun is not None:
        w.state[3:6] = u_fun(X, Y, Z)
    if A_fun is not None:
        w.state[0:3] = A_fun(X, Y, Z)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    return w, F


def _rhs(w, F):
    R, _ = O.rhs(F, 0.0, w.grid, w.params, None)
    return R


LNRHO = lambda X, Y, Z: 0.4 * np.sin(X + 2 * Y) + 0.3 * np.cos(Z - X) + 0.2 * np.sin(Y + Z)


def _u_fun(X, Y, Z):
    # a compressive and a rotational part in every component
    return np.stack([0.10 * np.sin(Y + Z) + 0.06 * np.cos(X),
                     0.08 * np.cos(X - 2 * Z) + 0.05 * np.sin(Y - X),
                     0.07 * np.sin(X + Y) + 0.04 * np.cos(2 * Z + Y)])


def _A_fun(X, Y, Z):
    return np.stack([0.08 * np.sin(Y + Z), 0.06 * np.cos(2 * X - Z), 0.07 * np.sin(X + Y)])


def _converges(errs, scale):
    """Sixth order: the error drops by ~2^6 per doubling (the pre-asymptotic
    ratio of these fields at 16 -> 32 is within [2^5, 2^7])."""
    assert errs[1] < 1e-4 * scale, (errs, scale)
    assert 2 ** 5 < errs[0] / errs[1] < 2 ** 7, errs


def test_mass_diffusion_equals_laplacian_of_rho_over_rho():
    # u = 0: d ln rho/dt is the mass diffusion alone, D_rho lap(rho)/rho
    Drho = 0.7
    (X, Y, Z), d = _spectral_ops(64)
    rho = np.exp(LNRHO(X, Y, Z))
    ref_full = Drho * sum(d(d(rho, i), i) for i in range(3)) / rho
    errs = []
    for n in (16, 32):
        w, F = _box(n, LNRHO, D_rho=Drho)
        R = _rhs(w, F)
        s = 64 // n
        errs.append(np.max(np.abs(R[6] - ref_full[::s, ::s, ::s])))
    _converges(errs, np.max(np.abs(ref_full)))


def test_mass_diffusion_gradient_term_is_not_a_laplacian_alone():
    # the |grad ln rho|^2 part is O(1) here: lap(ln rho) alone misses it
    (X, Y, Z), d = _spectral_ops(64)
    lr = LNRHO(X, Y, Z)
    rho = np.exp(lr)
    full = sum(d(d(rho, i), i) for i in range(3)) / rho
    lap = sum(d(d(lr, i), i) for i in range(3))
    assert np.max(np.abs(full - lap)) > 0.1 * np.max(np.abs(full))


def test_viscous_force_is_divergence_of_stress():
    # R_u(nu) - R_u(0) = div(2 rho nu S)/rho, S the traceless rate of strain
    nu = 0.9
    (X, Y, Z), d = _spectral_ops(64)
    u = _u_fun(X, Y, Z)
    rho = np.exp(LNRHO(X, Y, Z))
    G = [[d(u[i], j) for j in range(3)] for i in range(3)]   # G[i][j] = d_j u_i
    divu = G[0][0] + G[1][1] + G[2][2]
    S = [[0.5 * (G[i][j] + G[j][i]) - (divu / 3.0 if i == j else 0.0) for j in range(3)]
         for i in range(3)]
    ref_full = [sum(d(2.0 * rho * nu * S[i][j], j) for j in range(3)) / rho for i in range(3)]
    scale = max(np.max(np.abs(r)) for r in ref_full)
    errs = []
    for n in (16, 32):
        w1, F1 = _box(n, LNRHO, _u_fun, nu=nu)
        w0, F0 = _box(n, LNRHO, _u_fun, nu=0.0)
        visc = _rhs(w1, F1)[3:6] - _rhs(w0, F0)[3:6]
        s = 64 // n
        errs.append(max(np.max(np.abs(visc[i] - ref_full[i][::s, ::s, ::s])) for i in range(3)))
    _converges(errs, scale)


def test_viscous_density_term_is_significant():
    # with uniform density the 2 S.grad ln rho term vanishes; the test above
    # uses a density whose term is a sizeable part of the force
    nu = 0.9
    (X, Y, Z), d = _spectral_ops(64)
    u = _u_fun(X, Y, Z)
    lr = LNRHO(X, Y, Z)
    G = [[d(u[i], j) for j in range(3)] for i in range(3)]
    divu = G[0][0] + G[1][1] + G[2][2]
    S = [[0.5 * (G[i][j] + G[j][i]) - (divu / 3.0 if i == j else 0.0) for j in range(3)]
         for i in range(3)]
    dens = [2.0 * nu * sum(S[i][j] * d(lr, j) for j in range(3)) for i in range(3)]
    rest = [nu * sum(d(d(u[i], j), j) for j in range(3)) for i in range(3)]
    assert max(np.max(np.abs(a)) for a in dens) > 0.2 * max(np.max(np.abs(b)) for b in rest)


def test_lorentz_force_with_nonuniform_density():
    # u = 0, eta = nu = 0: R_u(A) - R_u(A = 0) = J x B / rho
    Bext = (0.6, -0.3, 0.5)
    mu0 = 1.0
    (X, Y, Z), d = _spectral_ops(64)
    A = _A_fun(X, Y, Z)
    rho = np.exp(LNRHO(X, Y, Z))
    B = [d(A[2], 1) - d(A[1], 2) + Bext[0], d(A[0], 2) - d(A[2], 0) + Bext[1],
         d(A[1], 0) - d(A[0], 1) + Bext[2]]
    J = [(d(B[2], 1) - d(B[1], 2)) / mu0, (d(B[0], 2) - d(B[2], 0)) / mu0,
         (d(B[1], 0) - d(B[0], 1)) / mu0]
    ref_full = [(J[1] * B[2] - J[2] * B[1]) / rho, (J[2] * B[0] - J[0] * B[2]) / rho,
                (J[0] * B[1] - J[1] * B[0]) / rho]
    scale = max(np.max(np.abs(r)) for r in ref_full)
    errs = []
    for n in (16, 32):
        w1, F1 = _box(n, LNRHO, A_fun=_A_fun, Bext=Bext)
        w0, F0 = _box(n, LNRHO, Bext=Bext)
        lor = _rhs(w1, F1)[3:6] - _rhs(w0, F0)[3:6]
        s = 64 // n
        errs.append(max(np.max(np.abs(lor[i] - ref_full[i][::s, ::s, ::s])) for i in range(3)))
    _converges(errs, scale)


# ---------------------------------------------------------------------------
# time-step limits not covered by the advective and viscous pins
# ---------------------------------------------------------------------------

def _uniform_corona(n=8, T=10 ** 6.3, rho=1e4):
    """Periodic box at rest, uniform T and rho, the coronal loss table on,
    every other process off (code units of the stratified boxes)."""
    w = W.periodic_box(n, amp_A=0.0, amp_u=0.0, eta=0.0, nu=0.0)
    lnT_tab, lnL_tab = W.rad_table_code_units()
    w.params.update(R=W.coronal_params(10.0)["R"], rad_lnT=lnT_tab, rad_lnL=lnL_tab,
                    T_rad_lo=1e4, T_rad_hi=2e4)
    w.state[6] = math.log(rho)
    w.state[7] = math.log(T)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    return w, F, lnL_tab


def test_cfl_radiative_limit_closed_form():
    # T at the breakpoint 10^6.3 K (above the cut): Lambda~ is the table
    # value there, and dt = c_adv rho c_v T / (rho^2 Lambda~)
    T, rho = 10 ** 6.3, 1e4
    w, F, lnL_tab = _uniform_corona(T=T, rho=rho)
    p = w.params
    cv = p["R"] / (p["gamma"] - 1.0)
    lam = math.exp(lnL_tab[5])
    dt_rad = p["c_adv"] * rho * cv * T / (rho * rho * lam)
    h = L / 8
    dt_adv = p["c_adv"] * h / math.sqrt(p["gamma"] * p["R"] * T)
    assert dt_rad < 0.5 * dt_adv            # the radiative limit is the one taken
    assert abs(O.cfl_dt(F, w.grid, p) - dt_rad) <= 1e-14 * dt_rad


def test_cfl_radiative_limit_between_breakpoints_and_below_the_cut():
    # between two breakpoints ln Lambda~ is linear in ln T; below T_rad_lo
    # there is no loss and the advective limit is taken
    lnT_tab, lnL_tab = W.rad_table_code_units()
    a = 0.3
    lnT = (1 - a) * lnT_tab[5] + a * lnT_tab[6]
    T, rho = math.exp(lnT), 2e4
    w, F, _ = _uniform_corona(T=T, rho=rho)
    p = w.params
    cv = p["R"] / (p["gamma"] - 1.0)
    lam = math.exp((1 - a) * lnL_tab[5] + a * lnL_tab[6])
    dt_rad = p["c_adv"] * rho * cv * T / (rho * rho * lam)
    assert dt_rad < 0.5 * p["c_adv"] * (L / 8) / math.sqrt(p["gamma"] * p["R"] * T)
    assert abs(O.cfl_dt(F, w.grid, p) - dt_rad) <= 1e-13 * dt_rad
    w, F, _ = _uniform_corona(T=9e3, rho=rho)
    h = L / 8
    dt_adv = p["c_adv"] * h / math.sqrt(p["gamma"] * p["R"] * 9e3)
    assert abs(O.cfl_dt(F, w.grid, w.params) - dt_adv) <= 1e-14 * dt_adv


def test_cfl_nudging_limit():
    # c_nudge / max(tau_u, tau_A, tau_t) when it is the smallest limit
    w = W.periodic_box(8, amp_A=0.0, amp_u=0.0, eta=0.0, nu=0.0)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    h = L / 8
    dt_adv = 0.4 * h / math.sqrt(5.0 / 3.0)
    assert abs(O.cfl_dt(F, w.grid, w.params) - dt_adv) < 1e-15
    w.params.update(nc_tau=40.0, c_nudge=1.0)
    assert abs(O.cfl_dt(F, w.grid, w.params) - 1.0 / 40.0) < 1e-17
    # solar boundaries: the larger of the two nudging rates sets the limit
    wq = W.small_stratified(nx=8, ny=8, nz=12, Lxy=8.0, z1=10.0, nbip=1)
    p = W.base_params()
    p.update(R=wq.params["R"], z_s=8.0, z_t=10.0, tau_u=300.0, tau_A=900.0, c_nudge=1.0)
    wq.params = p
    wq.state[0:6] = 0.0
    wq.state[7] = math.log(1e4)
    Fq = O.from_compact(wq.state)
    O.fill_ghosts(Fq, wq.grid, p, wq.lnrho0_z)
    assert abs(O.cfl_dt(Fq, wq.grid, p) - 1.0 / 900.0) < 1e-17
