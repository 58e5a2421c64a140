"""Seeded synthetic workloads for the coronal MHD step.

This module only builds inputs: grids, parameter sets, 1-D background
profiles, initial states and photospheric driver targets.  It contains no
part of the time step itself (no stencils, no right-hand side, no boundary
rules, no integrator).  Both the CPU oracle and the GPU library receive the
arrays produced here, unchanged.

Units for the stratified boxes ("code units"): length 1 Mm, velocity 1 km/s,
time 1 ks, density 1e-12 kg/m^3, temperature 1 K, mu0 = 1, so that the unit of
the magnetic field is sqrt(mu0_SI * 1e-12) * 1e3 T = 1.121e-6 T.

The stratified boxes stand in for the paper's Hinode-driven active region
(Sect. 2.1-2.3: observed magnetograms and a granulation driver); no observed
data exists here, so bipoles built in Fourier space and a random solenoidal
velocity field take their place.

State layout returned by every builder: float64 array [8, nz+6, ny, nx], field
order Ax, Ay, Az, ux, uy, uz, lnrho, lnT, x fastest.  z carries three ghost
planes on each side; x and y are periodic and carry no ghosts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NGHOST = 3
FIELDS = ("Ax", "Ay", "Az", "ux", "uy", "uz", "lnrho", "lnT")

# --- physical constants (SI) -------------------------------------------------
K_B = 1.380649e-23
M_P = 1.67262192e-27
MU0_SI = 4e-7 * math.pi
MU_MEAN = 0.6                     # mean molecular weight (paper silent)

# --- code units ---------------------------------------------------------------
U_L = 1e6        # m
U_V = 1e3        # m/s
U_T = U_L / U_V  # s  (1 ks)
U_RHO = 1e-12    # kg/m^3
U_B = math.sqrt(MU0_SI * U_RHO) * U_V          # T
U_Q = U_RHO * U_V ** 2 / U_T                   # W/m^3 (volumetric heating)

# Optically thin loss function: breakpoints (log10 T [K], log10 Lambda
# [erg cm^3 s^-1]) of a continuous piecewise power law modelled on the
# classic RTV fit.  Only smoothness matters for the tests; the numbers are
# input data.
RAD_TABLE_LOG10 = (
    (4.3, -21.85), (4.6, -21.80), (4.9, -21.20), (5.4, -21.20),
    (5.75, -21.90), (6.3, -21.93), (7.0, -22.40),
)


def rad_table_code_units():
    """(ln T, ln Lambda~) breakpoints with n_e = n_H = rho/m_p folded in,
    so that Q_rad = rho^2 * exp(ln Lambda~) in code units."""
    fold = (U_RHO / M_P) ** 2 / U_Q     # converts rho_code^2 * Lambda_SI to Q_code
    lnT = np.array([a * math.log(10.0) for a, _ in RAD_TABLE_LOG10])
    lnL = np.array([math.log(fold * 1e-13 * 10.0 ** b) for _, b in RAD_TABLE_LOG10])
    return lnT, lnL


@dataclass
class Workload:
    name: str
    grid: dict
    params: dict
    lnrho0_z: np.ndarray          # [nz+6] background ln rho at z_k, k=-3..nz+2
    lnT0_z: np.ndarray            # [nz+6] background ln T
    state: np.ndarray             # [8, nz+6, ny, nx]
    uh_target: np.ndarray | None = None   # [2, ny, nx] driver u*
    ah_target: np.ndarray | None = None   # [2, ny, nx] A_h* (nudging target)
    bz_bottom: np.ndarray | None = None   # [ny, nx]   B_z at z=0 (input of A_h*)
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        g = self.grid
        return (g["nz"], g["ny"], g["nx"])


# ---------------------------------------------------------------------------
# grids and parameter sets
# ---------------------------------------------------------------------------

def grid_dict(nx, ny, nz, Lx, Ly, z0, z1, zbc):
    return dict(nx=int(nx), ny=int(ny), nz=int(nz), Lx=float(Lx), Ly=float(Ly),
                z0=float(z0), z1=float(z1), zbc=zbc)


def z_coords(grid):
    """z_k for k=-3..nz+2 and the spacing (uniform; solar z is
    vertex-centred), or the given heights and None on a non-uniform grid."""
    if "z" in grid:
        return np.asarray(grid["z"], dtype=float), None
    nz = grid["nz"]
    if grid["zbc"] == "solar":
        dz = (grid["z1"] - grid["z0"]) / (nz - 1)
    else:
        dz = (grid["z1"] - grid["z0"]) / nz
    k = np.arange(-NGHOST, nz + NGHOST)
    return grid["z0"] + k * dz, dz


def base_params():
    """Every parameter, all physics off."""
    return dict(gamma=5.0 / 3.0, R=1.0, mu0=1.0, eta=0.0, nu=0.0, D_rho=0.0,
                kappa0=0.0, g_z=0.0, Bext=(0.0, 0.0, 0.0), B_floor=1e-8,
                eta_s=0.0, chi_s=0.0, chi_rho=0.0, z_s=0.0, z_t=1.0,
                tau_u=0.0, tau_A=0.0, t_ramp=0.0, f_bot=0.2,
                rad_lnT=np.zeros(0), rad_lnL=np.zeros(0),
                T_rad_lo=1e4, T_rad_hi=2e4,
                nc_tau=0.0, nc_lnrho_magn=8.0, nc_lnrho_width=2.0, nc_z_max=3.0,
                nc_z_width=0.3,
                c_adv=0.4, c_diff=0.12, c_nudge=1.0)


def coronal_params(z1):
    """Stratified-box physics in code units (paper silent on most values)."""
    p = base_params()
    lnT, lnL = rad_table_code_units()
    p.update(
        R=K_B / (MU_MEAN * M_P) / U_V ** 2,   # 0.01376
        eta=1.0, nu=1.0,                       # 1e9 m^2/s
        D_rho=8e6 / (U_L * U_V),               # 8e6 m^2/s (Sect. 2.5)
        kappa0=1e-11 / (U_RHO * U_V ** 3 * U_L),  # 1e-11 SI -> 1e-14 code
        g_z=-274.0,
        B_floor=1e-4 / U_B,                    # 1 G
        eta_s=1.0, chi_s=1.0, chi_rho=1.0,     # swamp diffusivities
        z_s=z1 - 5.0, z_t=z1,                  # swamp over the top 5 Mm
        tau_u=0.5 * U_T,                       # 0.5 s^-1 (Sect. 2.3)
        tau_A=U_T / 300.0,                     # one granule lifetime
        t_ramp=60.0 / U_T,                     # one minute
        f_bot=0.2,
        rad_lnT=lnT, rad_lnL=lnL,
        T_rad_lo=1e4, T_rad_hi=2e4,
    )
    return p


# ---------------------------------------------------------------------------
# initial-condition helpers (input synthesis only)
# ---------------------------------------------------------------------------

def _kgrid(nx, ny, Lx, Ly):
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=Lx / nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=Ly / ny)
    KX, KY = np.meshgrid(kx, ky)          # [ny, nx]
    nyq = np.zeros((ny, nx), dtype=bool)
    nyq[:, nx // 2] = True
    nyq[ny // 2, :] = True
    return KX, KY, nyq


def bipole_field(nx, ny, Lx, Ly, nbip, seed, B0, sigma, sep):
    """B_z(x,y) made of nbip balanced Gaussian bipoles, built from the Fourier
    series of periodised Gaussians: exactly periodic, zero net flux, no
    Nyquist content.  Returns the real field [ny, nx]."""
    rng = np.random.default_rng(seed)
    KX, KY, nyq = _kgrid(nx, ny, Lx, Ly)
    coef = np.zeros((ny, nx), dtype=complex)
    env = 2 * np.pi * sigma ** 2 / (Lx * Ly) * np.exp(-0.5 * (KX ** 2 + KY ** 2) * sigma ** 2)
    for _ in range(nbip):
        cx, cy = rng.uniform(0, Lx), rng.uniform(0, Ly)
        th = rng.uniform(0, np.pi)
        dx, dy = 0.5 * sep * math.cos(th), 0.5 * sep * math.sin(th)
        for sgn, px, py in ((+1, cx + dx, cy + dy), (-1, cx - dx, cy - dy)):
            coef += sgn * env * np.exp(-1j * (KX * px + KY * py))
    coef[0, 0] = 0.0
    coef[nyq] = 0.0
    bz = np.real(np.fft.ifft2(coef) * (nx * ny))
    # peak normalisation to B0
    return bz * (B0 / np.max(np.abs(bz)))


def potential_A_from_bz(bz, Lx, Ly, z):
    """Initial potential field above z=0: A_h whose curl is bz at z=0,
    continued upward as a decaying potential field.  Returns [2, nz, ny, nx]
    for the heights z (1-D array).  Input synthesis for the initial state."""
    ny, nx = bz.shape
    KX, KY, nyq = _kgrid(nx, ny, Lx, Ly)
    K2 = KX ** 2 + KY ** 2
    K2[0, 0] = 1.0
    B = np.fft.fft2(bz)
    ax_hat = 1j * KY * B / K2
    ay_hat = -1j * KX * B / K2
    ax_hat[0, 0] = ay_hat[0, 0] = 0.0
    ax_hat[nyq] = ay_hat[nyq] = 0.0
    K = np.sqrt(KX ** 2 + KY ** 2)
    out = np.empty((2, len(z), ny, nx))
    for i, zz in enumerate(z):
        decay = np.exp(-K * max(zz, 0.0))
        out[0, i] = np.real(np.fft.ifft2(ax_hat * decay))
        out[1, i] = np.real(np.fft.ifft2(ay_hat * decay))
    return out


def solenoidal_uh(nx, ny, Lx, Ly, seed, rms, ell):
    """Random divergence-free horizontal velocity with a Gaussian spectrum of
    correlation length ell, renormalised to the given rms.  [2, ny, nx]"""
    rng = np.random.default_rng(seed)
    KX, KY, nyq = _kgrid(nx, ny, Lx, Ly)
    K = np.sqrt(KX ** 2 + KY ** 2)
    psi = (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx)))
    psi *= np.exp(-0.5 * (K * ell) ** 2)
    psi[0, 0] = 0.0
    psi[nyq] = 0.0
    ux = np.real(np.fft.ifft2(1j * KY * psi))
    uy = np.real(np.fft.ifft2(-1j * KX * psi))
    s = math.sqrt(np.mean(ux ** 2 + uy ** 2))
    return np.stack([ux, uy]) * (rms / s)


def tanh_T0(z, T_lo=4e3, T_hi=1e6, z_tr=2.0, w_tr=0.5):
    return T_lo + (T_hi - T_lo) * 0.5 * (1.0 + np.tanh((z - z_tr) / w_tr))


def hydrostatic_lnrho(z, T0fun, R, g_z, rho_bottom, nsub=64):
    """ln rho0(z) of an atmosphere in hydrostatic balance with temperature
    T0fun(z): d ln p / dz = g_z / (R T0), p = rho R T, ln p fixed at z=0.
    Composite 4-point Gauss-Legendre on nsub sub-intervals per cell."""
    xg, wg = np.polynomial.legendre.leggauss(4)
    lnp0 = math.log(rho_bottom * R * T0fun(np.array([0.0]))[0])
    i0 = int(np.argmin(np.abs(z)))
    assert abs(z[i0]) < 1e-12
    lnp = np.empty_like(z)
    lnp[i0] = lnp0

    def integral(a, b):
        edges = np.linspace(a, b, nsub + 1)
        tot = 0.0
        for lo, hi in zip(edges[:-1], edges[1:]):
            mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
            s = mid + half * xg
            tot += half * np.sum(wg * g_z / (R * T0fun(s)))
        return tot

    for i in range(i0 + 1, len(z)):
        lnp[i] = lnp[i - 1] + integral(z[i - 1], z[i])
    for i in range(i0 - 1, -1, -1):
        lnp[i] = lnp[i + 1] - integral(z[i], z[i + 1])
    return lnp - math.log(R) - np.log(T0fun(z))


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def periodic_box(n=16, seed_A=0, seed_u=1, amp_A=1e-2, amp_u=1e-3, eta=1e-3, nu=1e-3,
                 nmodes=4, Bext=(0.0, 0.0, 0.0)):
    """Fully periodic box of side 2*pi, uniform ln rho = ln T = 0, A and u sums
    of random sine modes (integer wave vectors in [-2,2]^3 without 0)."""
    L = 2 * np.pi
    grid = grid_dict(n, n, n, L, L, 0.0, L, "periodic")
    p = base_params()
    p.update(eta=eta, nu=nu, Bext=tuple(float(b) for b in Bext))
    z, dz = z_coords(grid)
    x = np.arange(n) * (L / n)
    Z, Y, X = np.meshgrid(z, x, x, indexing="ij")
    state = np.zeros((8, n + 6, n, n))

    def modes(seed, amp):
        rng = np.random.default_rng(seed)
        out = np.zeros((3,) + Z.shape)
        for _ in range(nmodes):
            while True:
                k = rng.integers(-2, 3, size=3)
                if np.any(k != 0):
                    break
            e = rng.standard_normal(3)
            e /= np.linalg.norm(e)
            ph = rng.uniform(0, 2 * np.pi)
            s = np.sin(k[0] * X + k[1] * Y + k[2] * Z + ph)
            out += amp * e[:, None, None, None] * s[None]
        return out

    state[0:3] = modes(seed_A, amp_A)
    state[3:6] = modes(seed_u, amp_u)
    return Workload(name=f"periodic{n}", grid=grid, params=p,
                    lnrho0_z=np.zeros(n + 6), lnT0_z=np.zeros(n + 6), state=state)


def enable_newton_cooling(w: "Workload", tau=0.5 * U_T):
    """Switch on the chromospheric Newtonian cooling (Sect. 3.1; tau_t =
    0.5 s^-1, cutoffs 8 natural-log orders below the photospheric density with
    a sine over the last 2, and 3 Mm with a sine over the top 0.3 Mm) with the
    workload's initial profiles as its reference stratification."""
    w.params.update(nc_tau=tau, nc_lnrho_magn=8.0, nc_lnrho_width=2.0, nc_z_max=3.0,
                    nc_z_width=0.3, nc_lnrho0_z=np.array(w.lnrho0_z),
                    nc_lnT0_z=np.array(w.lnT0_z))
    return w


def stretched_heights(nz, z0, d_lo, d_hi, k_c, width):
    """Heights z_k, k = -3..nz+2, of a grid whose spacing rises smoothly from
    d_lo to d_hi around plane index k_c (a tanh over `width` planes), in
    closed form: dz/dk = d_lo + (d_hi - d_lo) (1 + tanh((k - k_c)/width)) / 2."""
    k = np.arange(-NGHOST, nz + NGHOST, dtype=float)
    lc = lambda x: np.logaddexp(x, -x) - math.log(2.0)     # ln cosh, overflow-free
    return z0 + d_lo * k + 0.5 * (d_hi - d_lo) * (
        k + width * (lc((k - k_c) / width) - lc(-k_c / width)))


def stratified_box(nx, ny, nz, Lxy, z1, nbip, seed_bip, seed_u, name, t_ramp=None, z=None):
    """Stratified coronal box: tanh T0(z) 4e3 K -> 1e6 K at 2 Mm (width
    0.5 Mm), hydrostatic ln rho0 with rho(0) = 2.7e-4 kg/m^3, bottom B_z from
    seeded bipoles (peak 1 kG, sigma 2 Mm, separation 6 Mm) continued as a
    potential field, u = 0, driver u* solenoidal with rms 1 km/s and 1 Mm
    correlation length."""
    if z is not None:
        z1 = float(z[NGHOST + nz - 1])
    grid = grid_dict(nx, ny, nz, Lxy, Lxy, 0.0, z1, "solar")
    if z is not None:
        # non-uniform heights: z0, z1 are the bottom and top interior planes
        grid.update(z=np.asarray(z, dtype=float), z0=float(z[NGHOST]),
                    z1=float(z[NGHOST + nz - 1]))
        z1 = grid["z1"]
    p = coronal_params(z1)
    if t_ramp is not None:
        p["t_ramp"] = t_ramp
    z, dz = z_coords(grid)
    lnT0 = np.log(tanh_T0(z))
    lnrho0 = hydrostatic_lnrho(z, tanh_T0, p["R"], p["g_z"], 2.7e-4 / U_RHO)
    B0 = 0.1 / U_B
    bz = bipole_field(nx, ny, Lxy, Lxy, nbip, seed_bip, B0, 2.0, 6.0)
    state = np.zeros((8, nz + 6, ny, nx))
    state[0:2] = potential_A_from_bz(bz, Lxy, Lxy, z)
    state[6] = lnrho0[:, None, None]
    state[7] = lnT0[:, None, None]
    uh = solenoidal_uh(nx, ny, Lxy, Lxy, seed_u, 1.0, 1.0)
    ah = state[0:2, NGHOST].copy()
    return Workload(name=name, grid=grid, params=p, lnrho0_z=lnrho0, lnT0_z=lnT0,
                    state=state, uh_target=uh, ah_target=ah, bz_bottom=bz)


def small_stretched(nx=32, ny=32, nz=24, Lxy=20.0, nbip=2, seed_bip=2, seed_u=3, t_ramp=None):
    """Reduced stratified box on a non-uniform z grid: spacing 0.25 Mm up to
    ~2.5 Mm, rising to 1.5 Mm above (top ~22 Mm)."""
    z = stretched_heights(nz, 0.0, 0.25, 1.5, 10.0, 4.0)
    return stratified_box(nx, ny, nz, Lxy, None, nbip, seed_bip, seed_u,
                          f"stretch{nx}x{ny}x{nz}", t_ramp=t_ramp, z=z)


def strat512_stretched():
    """The 512 x 512 x 256 box on the paper's kind of z grid: 100 km spacing
    through the photosphere and chromosphere rising to 800 km in the corona
    (top ~141 Mm)."""
    z = stretched_heights(256, 0.0, 0.1, 0.8, 90.0, 20.0)
    return stratified_box(512, 512, 256, 50.0, None, 8, 2, 3, "strat512_stretched", z=z)


def strat64():
    return stratified_box(64, 64, 64, 50.0, 50.0, 8, 2, 3, "strat64")


def strat512():
    return stratified_box(512, 512, 256, 50.0, 50.0, 8, 2, 3, "strat512")


def adjoint128():
    w = stratified_box(128, 128, 64, 50.0, 50.0, 8, 2, 3, "adjoint128", t_ramp=0.0)
    g = w.grid
    bz_t = bipole_field(g["nx"], g["ny"], g["Lx"], g["Ly"], 8, 5, 0.1 / U_B, 2.0, 6.0)
    # target: potential-field B_z of the second bipole set at z = 10 Mm
    KX, KY, _ = _kgrid(g["nx"], g["ny"], g["Lx"], g["Ly"])
    K = np.sqrt(KX ** 2 + KY ** 2)
    w.extra["bz_target_z10"] = np.real(np.fft.ifft2(np.fft.fft2(bz_t) * np.exp(-K * 10.0)))
    w.extra["loss_z"] = 10.0
    return w


def ar1024():
    return stratified_box(1024, 1024, 256, 64.0, 50.0, 32, 11, 3, "ar1024")


def granulation_randoms(n: int, seed: int):
    """Random pools of the granulation driver: n uniforms in [0, 1) (birth
    positions) and 2n standard-normal draws truncated to [-1, 1] by rejection
    (lifetime and amplitude variations)."""
    rng = np.random.default_rng(seed)
    unif = rng.random(n)
    xi = np.empty(2 * n)
    k = 0
    while k < 2 * n:
        d = rng.standard_normal(4 * n)
        d = d[np.abs(d) <= 1.0][: 2 * n - k]
        xi[k:k + d.size] = d
        k += d.size
    return unif, xi


def driver_reseed(w: Workload, seed: int):
    """A fresh driver target for the same box (used every 10 steps)."""
    g = w.grid
    return solenoidal_uh(g["nx"], g["ny"], g["Lx"], g["Ly"], seed, 1.0, 1.0)


def small_stratified(nx=32, ny=32, nz=24, Lxy=20.0, z1=20.0, nbip=2, seed_bip=2, seed_u=3,
                     t_ramp=None):
    """Reduced stratified box for quick tests: same physics, smaller grid."""
    return stratified_box(nx, ny, nz, Lxy, z1, nbip, seed_bip, seed_u,
                          f"strat{nx}x{ny}x{nz}", t_ramp=t_ramp)


WORKLOADS = {
    "strat512_stretched": strat512_stretched,
    "periodic16": lambda: periodic_box(16),
    "strat64": strat64,
    "strat512": strat512,
    "adjoint128": adjoint128,
    "ar1024": ar1024,
}
