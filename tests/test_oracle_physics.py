"""Pins of the oracle's right-hand side, integrator and boundary rules against
closed forms, exact discrete solutions and convergence rates.

Each test names the part of the step it fixes; together they are meant to
catch a dropped term, a flipped sign or a transposed index anywhere in the
oracle (the paper gives no worked example of a full step).
"""
import math

import numpy as np
import pytest

from oracle import mhd as O
from paper_1908_08557_amd import workloads as W

NG = 3


def symbols(k, h):
    th = k * h
    kt = (45 * np.sin(th) - 9 * np.sin(2 * th) + np.sin(3 * th)) / (30 * h)
    kh2 = (49 / 18 - 3 * np.cos(th) + 0.3 * np.cos(2 * th) - np.cos(3 * th) / 45) / h ** 2
    return kt, kh2


def rk3_poly(Z):
    """Amplification of any 3-stage third-order RK for y' = M y: I + Z + Z^2/2 + Z^3/6."""
    I = np.eye(Z.shape[0], dtype=complex)
    return I + Z + Z @ Z / 2 + Z @ Z @ Z / 6


def ghosted(w):
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    return F


# ---------------------------------------------------------------------------
# linear waves: exact discrete evolution of single Fourier modes
# ---------------------------------------------------------------------------

def _linear_mode_setup(n, k, B0, U, eps, eta, nu, Drho):
    w = W.periodic_box(n, amp_A=0.0, amp_u=0.0, eta=eta, nu=nu, Bext=(B0, 0.0, 0.0))
    w.params["D_rho"] = Drho
    x = np.arange(n) * (2 * np.pi / n)
    rng = np.random.default_rng(11)
    q0 = eps * (rng.standard_normal(5) + 1j * rng.standard_normal(5))  # Az, uy, ux, lnrho, lnT
    e = np.exp(1j * k * x)[None, None, :]
    w.state[2] = np.real(q0[0] * e)
    w.state[4] = np.real(q0[1] * e)
    w.state[3] = U + np.real(q0[2] * e)
    w.state[6] = np.real(q0[3] * e)
    w.state[7] = np.real(q0[4] * e)
    return w, q0, e


def _linear_operator(k, h, B0, U, eta, nu, Drho, gamma, R=1.0, T0=1.0):
    kt, kh2 = symbols(k, h)
    ik = 1j * kt
    M = np.zeros((5, 5), dtype=complex)
    # Alfven pair (A_z, u_y): induction u x B and resistivity; Lorentz force and shear viscosity
    M[0, 0] = -U * ik - eta * kh2
    M[0, 1] = -B0
    M[1, 0] = B0 * kh2
    M[1, 1] = -U * ik - nu * kh2
    # sound triple (u_x, ln rho, ln T): pressure, compression, compressive viscosity, mass diffusion
    M[2, 2] = -U * ik - 4.0 / 3.0 * nu * kh2
    M[2, 3] = -R * T0 * ik
    M[2, 4] = -R * T0 * ik
    M[3, 2] = -ik
    M[3, 3] = -U * ik - Drho * kh2
    M[4, 2] = -(gamma - 1.0) * ik
    M[4, 4] = -U * ik
    return M


def test_alfven_wave_exact_discrete_phase():
    # P12: uniform rho, T, B_ext = B0 x, eta = nu = 0: the mode amplitude is
    # multiplied per step by the RK3 polynomial of dt * M (phase speed v_A k^/k)
    n, k, B0 = 16, 2, 1.3
    eps = 1e-10
    w, q0, e = _linear_mode_setup(n, k, B0, 0.0, eps, 0.0, 0.0, 0.0)
    F = ghosted(w)
    dt = O.cfl_dt(F, w.grid, w.params)
    nsteps = 10
    F2, _ = O.run(F, 0.0, dt, nsteps, w.grid, w.params, w.lnrho0_z)
    h = 2 * np.pi / n
    M = _linear_operator(k, h, B0, 0.0, 0.0, 0.0, 0.0, w.params["gamma"])
    q = np.linalg.matrix_power(rk3_poly(dt * M), nsteps) @ q0
    got_Az = O.interior(F2[2])[0, 0]
    got_uy = O.interior(F2[4])[0, 0]
    ref_Az = np.real(q[0] * e)[0, 0]
    ref_uy = np.real(q[1] * e)[0, 0]
    scale = np.max(np.abs(q[:2]))
    assert np.max(np.abs(got_Az - ref_Az)) < 1e-9 * scale
    assert np.max(np.abs(got_uy - ref_uy)) < 1e-9 * scale
    # the discrete phase speed tends to v_A: eigenvalues of M are +-i B0 k^
    kt, kh2 = symbols(k, h)
    ev = np.linalg.eigvals(M[:2, :2])
    assert np.allclose(sorted(ev.imag), [-B0 * math.sqrt(kh2), B0 * math.sqrt(kh2)], rtol=1e-13)


def test_sound_and_diffusion_modes_exact():
    # pressure gradient, compression in continuity and energy, compressive and
    # shear viscosity, resistivity and mass diffusion on single modes
    n, k, B0 = 16, 3, 0.7
    eta, nu, Drho = 2e-2, 3e-2, 1e-2
    eps = 1e-10
    w, q0, e = _linear_mode_setup(n, k, B0, 0.0, eps, eta, nu, Drho)
    F = ghosted(w)
    dt = O.cfl_dt(F, w.grid, w.params)
    F2 = O.rk3_step(F, 0.0, dt, w.grid, w.params, w.lnrho0_z)
    h = 2 * np.pi / n
    M = _linear_operator(k, h, B0, 0.0, eta, nu, Drho, w.params["gamma"])
    q = rk3_poly(dt * M) @ q0
    idx = (2, 4, 3, 6, 7)
    scale = np.max(np.abs(q))
    for j, c in enumerate(idx):
        got = O.interior(F2[c])[0, 0]
        ref = np.real(q[j] * e)[0, 0]
        assert np.max(np.abs(got - ref)) < 1e-9 * scale, c
    # fields that stay zero to first order
    for c in (0, 1, 5):
        assert np.max(np.abs(O.interior(F2[c]))) < 1e-15


def test_advection_by_uniform_flow():
    # -u.grad of every field and u x B of the induction equation with U x
    n, k, B0, U = 16, 2, 0.5, 0.4
    eps = 1e-7
    w, q0, e = _linear_mode_setup(n, k, B0, U, eps, 1e-2, 1e-2, 0.0)
    F = ghosted(w)
    dt = O.cfl_dt(F, w.grid, w.params)
    F2 = O.rk3_step(F, 0.0, dt, w.grid, w.params, w.lnrho0_z)
    h = 2 * np.pi / n
    M = _linear_operator(k, h, B0, U, 1e-2, 1e-2, 0.0, w.params["gamma"])
    q = rk3_poly(dt * M) @ q0
    scale = np.max(np.abs(q))
    for j, c in enumerate((2, 4, 3, 6, 7)):
        got = O.interior(F2[c])[0, 0] - (U if c == 3 else 0.0)
        ref = np.real(q[j] * e)[0, 0]
        assert np.max(np.abs(got - ref)) < 1e-5 * scale, c


def test_translation_equivariance_bitwise():
    # P6: integer periodic shift of the inputs shifts the outputs, bitwise
    w = W.periodic_box(16)
    F = ghosted(w)
    dt = O.cfl_dt(F, w.grid, w.params)
    out = O.to_compact(O.rk3_step(F, 0.0, dt, w.grid, w.params, w.lnrho0_z))
    shift = (3, -5, 7)   # z (interior), y, x
    s = w.state.copy()
    s[:, NG:-NG] = np.roll(s[:, NG:-NG], shift, axis=(1, 2, 3))
    w.state = s
    out2 = O.to_compact(O.rk3_step(ghosted(w), 0.0, dt, w.grid, w.params, w.lnrho0_z))
    ref = np.roll(out[:, NG:-NG], shift, axis=(1, 2, 3))
    assert np.array_equal(out2[:, NG:-NG], ref)


# ---------------------------------------------------------------------------
# heating terms on single modes
# ---------------------------------------------------------------------------

def test_viscous_and_ohmic_heating():
    n, k = 16, 2
    U, a = 0.3, 0.2
    eta, nu = 0.05, 0.07
    w = W.periodic_box(n, amp_A=0.0, amp_u=0.0, eta=eta, nu=nu)
    x = np.arange(n) * (2 * np.pi / n)
    w.state[4] = U * np.sin(k * x)[None, None, :]      # shear flow u_y(x)
    w.state[1] = a * np.sin(k * x)[None, None, :]      # A_y(x): B_z = d_x A_y
    F = ghosted(w)
    R, _ = O.rhs(F, 0.0, w.grid, w.params, None)
    h = 2 * np.pi / n
    kt, kh2 = symbols(k, h)
    cv = 1.0 / (w.params["gamma"] - 1.0)
    visc = nu * (U * kt * np.cos(k * x)) ** 2          # 2 rho nu S:S
    ohm = eta * (kh2 * a * np.sin(k * x)) ** 2         # eta (curl B)^2 / mu0
    ref = (visc + ohm) / cv
    assert np.max(np.abs(R[7] - ref[None, None, :])) < 1e-13 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# Spitzer conduction along B
# ---------------------------------------------------------------------------

def _spitzer_rhs(n, lnT_fun, Bext, A_fun=None, kappa0=1.0):
    w = W.periodic_box(n, amp_A=0.0, amp_u=0.0, Bext=Bext, eta=0.0, nu=0.0)
    w.params["kappa0"] = kappa0
    L = 2 * np.pi
    z, _ = W.z_coords(w.grid)
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    w.state[7] = lnT_fun(X, Y, Z)
    if A_fun is not None:
        w.state[0:3] = A_fun(X, Y, Z)
    F = ghosted(w)
    R, _ = O.rhs(F, 0.0, w.grid, w.params, None)
    cv = 1.0 / (w.params["gamma"] - 1.0)
    T = np.exp(O.interior(F[7]))
    return R[7] * cv * T, (X, Y, Z)        # rho = 1: Q_cond


def test_spitzer_zero_across_field():
    # P13(i): uniform B along x, T = T(y): no conduction (to round-off: the
    # 7-point D2 of a constant sums -490+540-54+4 rounded products)
    q, _ = _spitzer_rhs(16, lambda X, Y, Z: 0.4 * np.sin(Y), (1.0, 0.0, 0.0))
    qy, _ = _spitzer_rhs(16, lambda X, Y, Z: 0.4 * np.sin(Y), (0.0, 1.0, 0.0))
    assert np.max(np.abs(q)) < 1e-14 * np.max(np.abs(qy))


def test_spitzer_along_field_converges_sixth_order():
    # P13(ii): B along x, ln T = 0.3 sin(x): Q = d_x(kappa0 T^5/2 d_x T)
    errs = []
    for n in (16, 32):
        q, (X, Y, Z) = _spitzer_rhs(n, lambda X, Y, Z: 0.3 * np.sin(X), (1.0, 0.0, 0.0))
        x = X[NG:-NG, :, :]
        G = 0.3 * np.cos(x)
        H = -0.3 * np.sin(x)
        T = np.exp(0.3 * np.sin(x))
        ref = T ** 3.5 * (3.5 * G * G + H)
        errs.append(np.max(np.abs(q - ref)))
    assert 2 ** 5.5 < errs[0] / errs[1] < 2 ** 6.5


def test_spitzer_axis_permutation():
    # P13(iii): field and gradient along y give the transposed result of x
    qx, _ = _spitzer_rhs(16, lambda X, Y, Z: 0.3 * np.sin(2 * X), (1.0, 0.0, 0.0))
    qy, _ = _spitzer_rhs(16, lambda X, Y, Z: 0.3 * np.sin(2 * Y), (0.0, 1.0, 0.0))
    qz, _ = _spitzer_rhs(16, lambda X, Y, Z: 0.3 * np.sin(2 * Z), (0.0, 0.0, 1.0))
    assert np.max(np.abs(qx - np.swapaxes(qy, 1, 2))) < 1e-14
    assert np.max(np.abs(qx - np.swapaxes(qz, 0, 2))) < 1e-14


def _spectral_conduction(nref, lnT_fun, A_fun, Bext, Bfloor):
    """div(T^5/2 b (b.grad T)) with b = B/sqrt(B.B + floor^2), B = curl A + Bext,
    all derivatives spectral on an nref^3 periodic grid (independent route)."""
    L = 2 * np.pi
    x = np.arange(nref) * (L / nref)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    k = np.fft.fftfreq(nref, d=1.0 / nref)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    Kv = (KX, KY, KZ)

    def d(f, i):
        return np.real(np.fft.ifftn(1j * Kv[i] * np.fft.fftn(f)))

    A = A_fun(X, Y, Z)
    B = [d(A[2], 1) - d(A[1], 2) + Bext[0], d(A[0], 2) - d(A[2], 0) + Bext[1],
         d(A[1], 0) - d(A[0], 1) + Bext[2]]
    Bn = np.sqrt(B[0] ** 2 + B[1] ** 2 + B[2] ** 2 + Bfloor ** 2)
    b = [Bi / Bn for Bi in B]
    T = np.exp(lnT_fun(X, Y, Z))
    gT = [d(T, i) for i in range(3)]
    bg = b[0] * gT[0] + b[1] * gT[1] + b[2] * gT[2]
    F = [T ** 2.5 * b[i] * bg for i in range(3)]
    return d(F[0], 0) + d(F[1], 1) + d(F[2], 2)


def test_spitzer_with_curved_field_matches_spectral_divergence():
    # the curvature terms (b.grad B).grad T and the d|B| term of the expanded
    # form, against a spectral divergence of the flux: error drops ~2^6
    lnT_fun = lambda X, Y, Z: 0.2 * np.sin(X + 2 * Y) + 0.15 * np.cos(Z - Y)

    def A_fun(X, Y, Z):
        return np.stack([0.08 * np.sin(Y + Z), 0.06 * np.cos(2 * X - Z), 0.07 * np.sin(X + Y)])

    Bext = (0.6, -0.3, 0.5)
    ref_full = _spectral_conduction(64, lnT_fun, A_fun, Bext, 1e-8)
    errs = []
    for n in (16, 32):
        q, _ = _spitzer_rhs(n, lnT_fun, Bext, A_fun)
        s = 64 // n
        ref = ref_full[::s, ::s, ::s]
        errs.append(np.max(np.abs(q - ref)))
    assert errs[1] < 1e-4 * np.max(np.abs(ref_full))
    assert errs[0] / errs[1] > 2 ** 5


# ---------------------------------------------------------------------------
# radiation and its cut
# ---------------------------------------------------------------------------

def test_radiation_table_breakpoints_and_continuity():
    lnT, lnL = W.rad_table_code_units()
    got = O.ln_lambda(lnT.copy(), lnT, lnL)
    assert np.allclose(got, lnL, rtol=0, atol=1e-13)
    eps = 1e-9
    lo = O.ln_lambda(lnT[1:-1] - eps, lnT, lnL)
    hi = O.ln_lambda(lnT[1:-1] + eps, lnT, lnL)
    assert np.max(np.abs(hi - lo)) < 1e-8
    # flat outside
    assert O.ln_lambda(np.array([lnT[0] - 1.0]), lnT, lnL)[0] == lnL[0]
    assert O.ln_lambda(np.array([lnT[-1] + 1.0]), lnT, lnL)[0] == lnL[-1]
    # midpoint of a segment is the mean of the end values (power law in T)
    mid = 0.5 * (lnT[2] + lnT[3])
    assert abs(O.ln_lambda(np.array([mid]), lnT, lnL)[0] - 0.5 * (lnL[2] + lnL[3])) < 1e-13


def test_radiation_cut_is_c1():
    lo, hi = 1e4, 2e4
    a, b = math.log(lo), math.log(hi)
    f = lambda x: O.rad_cut(np.array([x]), lo, hi)[0]
    assert f(a) == 0.0 and f(b) == 1.0 and f(a - 1) == 0.0 and f(b + 1) == 1.0
    e = 1e-6
    for x in (a, b):
        left = (f(x) - f(x - e)) / e
        right = (f(x + e) - f(x)) / e
        assert abs(left) < 1e-5 and abs(right) < 1e-5
    assert abs(f(0.5 * (a + b)) - 0.5) < 1e-15


@pytest.mark.parametrize("T0", [8e3, 1.5e4, 5e4, 3e5, 2e7])
def test_radiation_rhs_term(T0):
    # uniform plasma: d ln T/dt = -rho^2 Lambda(T) W(T) / (rho c_v T), with the
    # table flat below its first and above its last breakpoint
    w = W.periodic_box(8, amp_A=0.0, amp_u=0.0)
    lnT, lnL = W.rad_table_code_units()
    w.params.update(rad_lnT=lnT, rad_lnL=lnL)
    rho0 = 2.0
    w.state[6] = math.log(rho0)
    w.state[7] = math.log(T0)
    F = ghosted(w)
    R, _ = O.rhs(F, 0.0, w.grid, w.params, None)
    x = math.log(T0)
    if x < lnT[0]:
        lam = lnL[0]
    elif x >= lnT[-1]:
        lam = lnL[-1]
    else:
        i = int(np.searchsorted(lnT, x, side="right")) - 1
        lam = lnL[i] + (lnL[i + 1] - lnL[i]) * (x - lnT[i]) / (lnT[i + 1] - lnT[i])
    s = min(1.0, max(0.0, (x - math.log(1e4)) / (math.log(2e4) - math.log(1e4))))
    wcut = 3 * s * s - 2 * s ** 3
    cv = 1.0 / (w.params["gamma"] - 1.0)
    ref = -rho0 ** 2 * math.exp(lam) * wcut / (rho0 * cv * T0)
    if ref == 0.0:
        assert np.max(np.abs(R[7])) == 0.0
    else:
        assert np.allclose(R[7], ref, rtol=1e-13, atol=0)


# ---------------------------------------------------------------------------
# nudging, integrator, hydrostatics (solar boundaries)
# ---------------------------------------------------------------------------

def _quiet_solar(nx=8, ny=8, nz=12, T0=1e4, g=0.0):
    """Solar box with uniform T, hydrostatic (linear) ln rho, everything off."""
    w = W.small_stratified(nx=nx, ny=ny, nz=nz, Lxy=8.0, z1=10.0, nbip=1)
    p = W.base_params()
    p.update(R=w.params["R"], g_z=g, kappa0=0.0, eta=0.0, nu=0.0)
    p.update(z_s=8.0, z_t=10.0)
    w.params = p
    z, dz = W.z_coords(w.grid)
    lnr = 2.0 + g * z / (p["R"] * T0)
    w.lnrho0_z = lnr
    w.lnT0_z = np.full_like(z, math.log(T0))
    w.state[:] = 0.0
    w.state[6] = lnr[:, None, None]
    w.state[7] = math.log(T0)
    w.uh_target[:] = 0.0
    w.ah_target[:] = 0.0
    return w


def test_nudging_exact_rk3_decay():
    # P11: u_h(k<=0) after n steps is u* (1 - P(-tau dt)^n); u = 0 above
    w = _quiet_solar()
    tau = 500.0
    w.params.update(tau_u=tau, t_ramp=0.0)
    ustar = np.array([0.7, -1.1])
    w.uh_target = np.ones((2, 8, 8)) * ustar[:, None, None]
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    F = ghosted(w)
    dt = 1e-3
    n = 7
    F2, _ = O.run(F, 0.0, dt, n, w.grid, w.params, w.lnrho0_z, drv)
    z = -tau * dt
    amp = (1 + z + z * z / 2 + z ** 3 / 6) ** n
    for c in (0, 1):
        for kz in range(0, NG + 1):     # planes k = -3..0
            got = F2[3 + c, kz, NG:-NG, NG:-NG]
            assert np.allclose(got, ustar[c] * (1 - amp), rtol=1e-13, atol=0)
        assert np.max(np.abs(F2[3 + c, NG + 1:NG + 12])) == 0.0
    assert np.max(np.abs(F2[5])) == 0.0


def test_ramp_scales_target():
    w = _quiet_solar()
    w.params.update(tau_u=10.0, t_ramp=0.06)
    w.uh_target = np.ones((2, 8, 8))
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    F = ghosted(w)
    R, Rg = O.rhs(F, 0.03, w.grid, w.params, drv)
    assert np.allclose(R[3, 0], 10.0 * 0.5, rtol=1e-15)
    assert np.allclose(Rg[0], 10.0 * 0.5, rtol=1e-15)
    R, Rg = O.rhs(F, 1.0, w.grid, w.params, drv)
    assert np.allclose(R[3, 0], 10.0, rtol=1e-15)


def test_magnetic_nudging_at_photosphere_only():
    w = _quiet_solar()
    w.params.update(tau_A=3.0)
    w.ah_target = np.ones((2, 8, 8)) * np.array([0.2, -0.4])[:, None, None]
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    F = ghosted(w)
    R, _ = O.rhs(F, 0.0, w.grid, w.params, drv)
    assert np.allclose(R[0, 0], 3.0 * 0.2) and np.allclose(R[1, 0], 3.0 * -0.4)
    assert np.max(np.abs(R[0:3, 1:])) == 0.0 and np.max(np.abs(R[2])) == 0.0


def test_isothermal_atmosphere_stays_at_rest():
    # P9: isothermal hydrostatic column, A = 0, radiation and nudging off,
    # D_rho = 0 (swamp, viscosity, resistivity and conduction on): u stays 0
    w = _quiet_solar(nz=16, g=-274.0, T0=2e4)
    w.params.update(eta=1.0, nu=1.0, kappa0=1e-14, eta_s=1.0, chi_s=1.0, chi_rho=1.0)
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    F = ghosted(w)
    dt = O.cfl_dt(F, w.grid, w.params)
    F2, _ = O.run(F, 0.0, dt, 100, w.grid, w.params, w.lnrho0_z, drv)
    cs = math.sqrt(w.params["gamma"] * w.params["R"] * 2e4)
    umax = max(np.max(np.abs(F2[c, NG:-NG])) for c in (3, 4, 5))
    assert umax / cs < 1e-12


def test_hydrostatic_residual_converges_sixth_order():
    # P10: resolved stratification (wide tanh): the momentum residual
    # -R T (d ln rho + d ln T) + g shrinks ~2^6 per doubling away from the
    # boundaries (near them the first-order ghost recursion dominates)
    def residual(nz):
        w = W.small_stratified(nx=8, ny=8, nz=nz, Lxy=8.0, z1=20.0, nbip=1)
        z, dz = W.z_coords(w.grid)
        Tf = lambda s: W.tanh_T0(s, T_lo=2e4, T_hi=1e5, z_tr=10.0, w_tr=3.0)
        lnr = W.hydrostatic_lnrho(z, Tf, w.params["R"], -274.0, 1.0, nsub=32)
        p = W.base_params()
        p.update(R=w.params["R"], g_z=-274.0)
        w.params = p
        w.lnrho0_z = lnr
        w.state[:] = 0.0
        w.state[6] = lnr[:, None, None]
        w.state[7] = np.log(Tf(z))[:, None, None]
        drv = dict(uh=w.uh_target * 0, ah=w.ah_target * 0)
        F = ghosted(w)
        R, _ = O.rhs(F, 0.0, w.grid, w.params, drv)
        zi = z[NG:-NG]
        sel = (zi > 5.0) & (zi < 15.0)
        return np.max(np.abs(R[5][sel]))

    e1, e2 = residual(33), residual(65)
    assert e1 / e2 > 2 ** 5.5


def test_lower_temperature_ghosts_hydrostatic():
    # eq. (8): linear T(z) below the photosphere; the recursion converges to
    # the analytic hydrostatic T at the ghost heights (first-order scheme)
    def ghost_err(nz):
        w = _quiet_solar(nz=nz, g=-274.0)
        z, dz = W.z_coords(w.grid)
        T0, alpha = 1e4, 0.05
        Tz = T0 * (1 + alpha * z)
        R = w.params["R"]
        lnp = (-274.0) / (R * T0 * alpha) * np.log(1 + alpha * z)
        w.lnrho0_z = lnp - np.log(R) - np.log(Tz)
        w.state[6] = w.lnrho0_z[:, None, None]
        w.state[7] = np.log(Tz)[:, None, None]
        F = ghosted(w)
        got = F[7, 0:NG, NG, NG]
        return np.max(np.abs(got - np.log(Tz[0:NG])))

    # the one-sided quadrature of d ln p/dz = g/(R T) leaves O(dz^2) per layer;
    # a wrong sign or a dropped term would leave O(dz/H) ~ 1
    errs = [ghost_err(n) for n in (21, 41, 81)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.25 * errs[0]
    assert errs[2] < 3e-3


def test_upper_and_velocity_ghost_rules():
    w = W.small_stratified(nx=16, ny=8, nz=12)
    rng = np.random.default_rng(3)
    w.state[3:6, NG:-NG] = rng.standard_normal(w.state[3:6, NG:-NG].shape)
    F = ghosted(w)
    nz = w.grid["nz"]
    kt = NG + nz - 1
    z, dz = W.z_coords(w.grid)
    R, g = w.params["R"], w.params["g_z"]
    for j in (1, 2, 3):
        assert np.array_equal(F[5, NG - j], -F[5, NG + j])          # u_z antisymmetric below
        assert np.array_equal(F[5, kt + j], -F[5, kt - j])          # and above
        assert np.array_equal(F[3, kt + j], F[3, kt - j])           # u_h symmetric above
        assert np.array_equal(F[7, kt + j], F[7, kt - j])           # eq. (11)
        ref = F[6, kt - j] + g * (2 * j * dz) / (R * np.exp(F[7, kt]))
        assert np.allclose(F[6, kt + j], ref, rtol=1e-15)            # eq. (13)
        assert np.all(F[6, NG - j] == w.lnrho0_z[NG - j])            # 'fg'


@pytest.mark.parametrize("mx,my", [(1, 0), (2, 3), (0, 3), (4, 4), (8, 1)])
def test_potential_field_ghosts_single_mode(mx, my):
    # P7/P8: a cos(k.r) at the top (bottom) plane -> a exp(-|k| j dz) cos(k.r)
    # above, a exp(+f_bot |k| j dz) cos(k.r) below, for every component
    nx, ny = 16, 8
    w = W.small_stratified(nx=nx, ny=ny, nz=10, Lxy=8.0, z1=6.0)
    Lx, Ly = w.grid["Lx"], w.grid["Ly"]
    x = np.arange(nx) * Lx / nx
    y = np.arange(ny) * Ly / ny
    Y, X = np.meshgrid(y, x, indexing="ij")
    kx, ky = 2 * np.pi * mx / Lx, 2 * np.pi * my / Ly
    kabs = math.hypot(kx, ky)
    mode = np.cos(kx * X + ky * Y + 0.4)
    amps = (0.3, -0.7, 1.1)
    for c in range(3):
        w.state[c] = amps[c] * mode[None]
    F = ghosted(w)
    _, dz = W.z_coords(w.grid)
    kt = NG + w.grid["nz"] - 1
    fb = w.params["f_bot"]
    for c in range(3):
        for j in (1, 2, 3):
            top = F[c, kt + j, NG:-NG, NG:-NG]
            bot = F[c, NG - j, NG:-NG, NG:-NG]
            assert np.max(np.abs(top - amps[c] * math.exp(-kabs * j * dz) * mode)) < 1e-14
            ref_b = amps[c] * math.exp(fb * kabs * j * dz) * mode
            assert np.max(np.abs(bot - ref_b)) < 1e-14 * max(1.0, np.max(np.abs(ref_b)))


def test_inverted_field_contrast_grows_with_depth():
    # Sect. 2.4: flux bundles get narrower and stronger below the photosphere
    w = W.small_stratified(nx=32, ny=32, nz=10)
    F = ghosted(w)
    h = O.spacings(w.grid)
    bz = []
    for k in (NG, NG - 1, NG - 2, NG - 3):
        Ay, Ax = F[1, k], F[0, k]
        b = O.d1(Ay, 1, h[0])[NG:-NG] - O.d1(Ax, 0, h[1])[:, NG:-NG]
        bz.append(np.max(np.abs(b)))
    assert bz[0] < bz[1] < bz[2] < bz[3]


# ---------------------------------------------------------------------------
# swamp
# ---------------------------------------------------------------------------

def test_swamp_weight_profile():
    zs, zt = 45.0, 50.0
    z = np.array([40.0, zs, 47.5, zt, 55.0])
    w, dw = O.swamp_weight(z, zs, zt)
    assert list(w) == [0.0, 0.0, 0.5, 1.0, 1.0]
    assert dw[1] == 0.0 and dw[3] == 0.0
    assert abs(dw[2] - 1.5 / (zt - zs)) < 1e-15
    # derivative matches a finite difference inside
    e = 1e-6
    zz = np.array([46.3])
    fd = (O.swamp_weight(zz + e, zs, zt)[0] - O.swamp_weight(zz - e, zs, zt)[0]) / (2 * e)
    assert abs(fd[0] - O.swamp_weight(zz, zs, zt)[1][0]) < 1e-8


def test_swamp_terms_on_horizontal_mode():
    # eqs. (18)-(20): the RHS difference from switching the swamp on equals
    # eta_s w lap(A) + e_z eta_s w' div A, chi_rho w lap(ln rho), chi_s w lap(ln T)
    nx = 16
    w = _quiet_solar(nx=nx, ny=8, nz=24)
    w.params.update(z_s=3.0, z_t=8.0)
    Lx = w.grid["Lx"]
    x = np.arange(nx) * Lx / nx
    k = 2 * np.pi * 2 / Lx
    s = np.sin(k * x)[None, None, :]
    w.state[0] = 0.3 * s           # A_x(x): div A = d_x A_x, lap A_x = -k^2 A_x
    w.state[6] = w.state[6] + 0.01 * s
    w.state[7] = w.state[7] + 0.02 * s
    drv = dict(uh=w.uh_target, ah=w.ah_target)
    F = ghosted(w)
    R0, _ = O.rhs(F, 0.0, w.grid, w.params, drv)
    w.params.update(eta_s=0.5, chi_rho=0.25, chi_s=0.75)
    R1, _ = O.rhs(F, 0.0, w.grid, w.params, drv)
    z, dz = W.z_coords(w.grid)
    zi = z[NG:-NG]
    wz, dwz = O.swamp_weight(zi, 3.0, 8.0)
    h = Lx / nx
    kt, kh2 = symbols(k, h)
    c = np.cos(k * x)[None, :]
    lap = -kh2 * np.sin(k * x)[None, :]
    for kk in range(4, 20):       # planes whose z-stencil sees no ghosts of A
        d = R1[:, kk] - R0[:, kk]
        assert np.allclose(d[0], 0.5 * wz[kk] * 0.3 * lap, atol=1e-14)
        assert np.allclose(d[2], 0.5 * dwz[kk] * 0.3 * kt * c, atol=1e-14)
        assert np.allclose(d[6], 0.25 * wz[kk] * 0.01 * lap, atol=1e-14)
        assert np.allclose(d[7], 0.75 * wz[kk] * 0.02 * lap, atol=1e-14)


# ---------------------------------------------------------------------------
# A_h* from B_z (eq. 7) and the CFL step
# ---------------------------------------------------------------------------

def test_ah_from_bz_spectral_curl():
    # P16: the spectral curl of A_h* reproduces B_z exactly; D1 converges
    nx, ny, L = 32, 16, 20.0
    bz = W.bipole_field(nx, ny, L, L * ny / nx, 2, 9, 1.0, 1.5, 3.0)
    ah = O.ah_from_bz(bz, L, L * ny / nx)
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=L / nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=(L * ny / nx) / ny)
    curl = np.real(np.fft.ifft2(1j * kx[None, :] * np.fft.fft2(ah[1])
                                - 1j * ky[:, None] * np.fft.fft2(ah[0])))
    assert np.max(np.abs(curl - bz)) < 1e-13 * np.max(np.abs(bz))


def test_cfl_dt_limits():
    w = W.periodic_box(8, amp_A=0.0, amp_u=0.0, eta=0.0, nu=0.0)
    w.state[3] = 0.5
    F = ghosted(w)
    h = 2 * np.pi / 8
    cs = math.sqrt(5.0 / 3.0)
    assert abs(O.cfl_dt(F, w.grid, w.params) - 0.4 * h / (0.5 + cs)) < 1e-15
    w.params.update(nu=10.0)
    assert abs(O.cfl_dt(F, w.grid, w.params) - 0.12 * h * h / 10.0) < 1e-15


@pytest.mark.parametrize("stretch", [False, True])
def test_patch_step_equals_whole_box_step(stretch):
    # the sampled full-size parity test rests on locality: one step of a
    # 25^3 periodic patch gives the whole-box step at its centre
    from parity_util import oracle_patch_centre
    if stretch:
        w = W.small_stretched(32, 32, 40, Lxy=20.0, nbip=2)
    else:
        w = W.small_stratified(32, 32, 40, Lxy=20.0, z1=30.0, nbip=2)
    F = O.from_compact(w.state)
    O.fill_ghosts(F, w.grid, w.params, w.lnrho0_z)
    dt = O.cfl_dt(F, w.grid, w.params)
    full = O.to_compact(O.rk3_step(F, 0.0, dt, w.grid, w.params, w.lnrho0_z,
                                   dict(uh=w.uh_target, ah=w.ah_target)))
    fmax = np.max(np.abs(full[:, NG:-NG]), axis=(1, 2, 3))
    for (k, j, i) in [(12, 5, 7), (20, 31, 0), (14, 16, 30)]:
        got = oracle_patch_centre(w, k, j, i, dt, 12)
        ref = full[:, NG + k, j, i]
        assert np.all(np.abs(got - ref) <= 1e-13 * np.maximum(fmax, 1e-30)), (k, j, i, got - ref)
