"""Plain FP64 CPU oracle for one RK3 time step of the coronal MHD model
(Bourdin 2019, "Driving solar coronal MHD simulations on high-performance
computers", arXiv:1908.08557).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this file; only the test suite, the smoke check and the CPU baseline of the
benchmark do.  It shares no code with the GPU path and uses its own array
layout: every field is a full [nz+6, ny+6, nx+6] array with materialised
ghost cells on all six faces (the GPU library stores no x/y ghosts).

Every operation is one plain numpy expression over whole arrays, written in the
order of the equations, in float64 (or complex128, for complex-step
derivatives: nothing here takes a real part or an absolute value of a state
quantity except to choose a branch).

What the paper fixes and what is a reading (the paper prints only the terms it
adds, "..." elsewhere):
  * State in vector potential A, velocity u, ln rho, ln T; B = curl A in the
    Weyl gauge (Sect. 2.4, eqs. 6-7).  Three ghost layers (Sect. 2.3-4.2).
  * Sixth-order centred first/second derivatives, mixed derivatives as the
    product of two first-derivative stencils, pure second derivatives with
    the 7-point stencil (reading; order from the problem statement).
  * Induction, momentum, continuity and energy equations in non-conservative
    form with constant eta and nu, Spitzer conduction along B (Sect. 3,
    Spitzer & Haerm), optically thin loss (Sect. 3, Cook et al.) - reading.
  * Photospheric nudging of u_h in layers 0..-3, eq. (5), with a linear
    switch-on ramp over the first minute (Sect. 2.3); magnetic nudging of A_h
    at the photosphere towards A_h* (Sect. 2.1, two distinct half times;
    the rate is a reading); A_h* from B_z through eq. (7).
  * Lower ghosts: inverted potential field with contrast factor f_bot
    (Sect. 2.4), density fixed to the initial profile ('fg', Sect. 2.5),
    u_z antisymmetric (closed), T from hydrostatic recursion eq. (8)
    (exponent read as dz*g/(R T) with signed g; the printed c_v identity is
    garbled).
  * Upper ghosts: potential field eqs. (16)-(17), T symmetric eq. (11),
    rho hydrostatic mirror eq. (13) with 1/gamma read as 1/R, u_z
    antisymmetric, u_h symmetric (closed, Sect. 4.1; u_h rule a reading).
  * Swamp layers eqs. (18)-(20) with the cubic step w(z) (Sect. 4.3).
  * Low-storage 2N RK3 of Williamson (1980) (reading; integrator not printed).
"""
from __future__ import annotations

import math

import numpy as np

NG = 3
# Williamson (1980) low-storage RK3 coefficients
RK_ALPHA = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK_BETA = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)
RK_C = (0.0, 1.0 / 3.0, 3.0 / 4.0)

AX, AY, AZ, UX, UY, UZ, LNRHO, LNT = range(8)


# ---------------------------------------------------------------------------
# grid helpers
# ---------------------------------------------------------------------------

class ZMetric:
    """Metric of a non-uniform z grid z_k = z(zeta = k) (reading: z is a smooth
    function of the plane index and the sixth-order stencils act in zeta):
    d/dz = m1 d/dzeta, d2/dz2 = m1^2 d2/dzeta2 + m2 d/dzeta, with
    m1 = 1/z', m2 = -z''/z'^3 and z', z'' the sixth-order differences of the
    heights themselves, at the interior planes k = 0..nz-1."""

    def __init__(self, z):
        z = np.asarray(z, dtype=float)
        zp = d1(z, 0, 1.0)
        zpp = d2(z, 0, 1.0)
        self.zp = zp
        self.m1 = 1.0 / zp
        self.m2 = -zpp / zp ** 3

    def col(self, a, ndim):
        return a.reshape((-1,) + (1,) * (ndim - 1))


def stretched(grid):
    return "z" in grid


def spacings(grid):
    """(dx, dy, dz).  Solar z is vertex-centred: z_0 = z0, z_{nz-1} = z1.  On
    a non-uniform z grid the third entry is its ZMetric."""
    dx = grid["Lx"] / grid["nx"]
    dy = grid["Ly"] / grid["ny"]
    if stretched(grid):
        return dx, dy, ZMetric(grid["z"])
    if grid["zbc"] == "solar":
        dz = (grid["z1"] - grid["z0"]) / (grid["nz"] - 1)
    else:
        dz = (grid["z1"] - grid["z0"]) / grid["nz"]
    return dx, dy, dz


def zk(grid):
    """Heights of the planes k = -3 .. nz+2."""
    if stretched(grid):
        return np.asarray(grid["z"], dtype=float)
    dz = spacings(grid)[2]
    return grid["z0"] + dz * np.arange(-NG, grid["nz"] + NG)


def swamp_weight(z, zs, zt):
    """Cubic step w(z): 0 below z_s, 1 above z_t, zero slope at both ends
    (Sect. 4.3).  Returns (w, dw/dz)."""
    s = np.clip((z - zs) / (zt - zs), 0.0, 1.0)
    w = s * s * (3.0 - 2.0 * s)
    inside = (z > zs) & (z < zt)
    dw = np.where(inside, 6.0 * s * (1.0 - s) / (zt - zs), 0.0)
    return w, dw


# ---------------------------------------------------------------------------
# layout conversion (test plumbing): compact [8,nz+6,ny,nx] <-> full ghosted
# ---------------------------------------------------------------------------

def from_compact(state):
    f, nzg, ny, nx = state.shape
    F = np.zeros((f, nzg, ny + 2 * NG, nx + 2 * NG), dtype=state.dtype)
    F[:, :, NG:-NG, NG:-NG] = state
    wrap_xy(F)
    return F


def to_compact(F):
    return np.ascontiguousarray(F[:, :, NG:-NG, NG:-NG])


def wrap_xy(F):
    """Periodic x and y ghosts, over every z plane (including z ghosts)."""
    n = F.shape[-1] - 2 * NG
    F[..., :NG] = F[..., n:n + NG]
    F[..., n + NG:] = F[..., NG:2 * NG]
    n = F.shape[-2] - 2 * NG
    F[..., :NG, :] = F[..., n:n + NG, :]
    F[..., n + NG:, :] = F[..., NG:2 * NG, :]


# ---------------------------------------------------------------------------
# Step 0: sixth-order centred stencils
# ---------------------------------------------------------------------------

def _shift(f, ax, o):
    """View of f shifted by o along ax, over the points where a +-3 stencil fits."""
    n = f.shape[ax]
    idx = [slice(None)] * f.ndim
    idx[ax] = slice(NG + o, n - NG + o)
    return f[tuple(idx)]


def d1(f, ax, h):
    """First derivative, 7-point, sixth order:
    [45 (f+1 - f-1) - 9 (f+2 - f-2) + (f+3 - f-3)] / (60 h).
    The result is 6 points shorter along ax.  h may be a ZMetric (z axis)."""
    if isinstance(h, ZMetric):
        return h.col(h.m1, f.ndim) * d1(f, ax, 1.0)
    s = lambda o: _shift(f, ax, o)
    return (45.0 * (s(1) - s(-1)) - 9.0 * (s(2) - s(-2)) + (s(3) - s(-3))) / (60.0 * h)


def d2(f, ax, h):
    """Second derivative, 7-point, sixth order:
    [-490 f0 + 270 (f+1 + f-1) - 27 (f+2 + f-2) + 2 (f+3 + f-3)] / (180 h^2).
    h may be a ZMetric (z axis)."""
    if isinstance(h, ZMetric):
        return (h.col(h.m1 * h.m1, f.ndim) * d2(f, ax, 1.0)
                + h.col(h.m2, f.ndim) * d1(f, ax, 1.0))
    s = lambda o: _shift(f, ax, o)
    return (-490.0 * s(0) + 270.0 * (s(1) + s(-1)) - 27.0 * (s(2) + s(-2))
            + 2.0 * (s(3) + s(-3))) / (180.0 * h * h)


def _crop(a, axes):
    idx = [slice(None)] * a.ndim
    for ax in axes:
        idx[ax] = slice(NG, a.shape[ax] - NG)
    return a[tuple(idx)]


# direction d (0=x, 1=y, 2=z) acts on array axis 2-d of a [z, y, x] field
def grad(f, d, h):
    """d_d f at interior points."""
    ax = 2 - d
    return d1(_crop(f, [a for a in range(3) if a != ax]), ax, h[d])


def hess(f, i, j, h):
    """d_i d_j f at interior points.  Pure: 7-point D2.  Mixed: D1 along i of
    D1 along j (36-point product stencil, uses edge and corner ghosts)."""
    if i == j:
        ax = 2 - i
        return d2(_crop(f, [a for a in range(3) if a != ax]), ax, h[i])
    ai, aj = 2 - i, 2 - j
    other = [a for a in range(3) if a not in (ai, aj)]
    inner = d1(_crop(f, other), aj, h[j])
    return d1(inner, ai, h[i])


def interior(f):
    return f[NG:-NG, NG:-NG, NG:-NG]


# ---------------------------------------------------------------------------
# 2-D Fourier filters of the photospheric and top planes (Sect. 4.2)
# ---------------------------------------------------------------------------

def _kabs_rfft(nx, ny, Lx, Ly):
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx, d=Lx / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=Ly / ny)
    return np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2)


def _filter_real(plane, factor):
    """Inverse-normalised 2-D transform pair with a real multiplier."""
    spec = np.fft.rfft2(plane)
    return np.fft.irfft2(spec * factor, s=plane.shape)


def kspace_filter(plane, factor):
    """Apply a real, even multiplier in k-space to a (possibly complex) plane;
    the real and imaginary parts are filtered separately (linear map)."""
    if np.iscomplexobj(plane):
        return _filter_real(plane.real, factor) + 1j * _filter_real(plane.imag, factor)
    return _filter_real(plane, factor)


def ah_from_bz(bz, Lx, Ly):
    """A_x, A_y with d_x A_y - d_y A_x = B_z (eq. 7), in Fourier space:
    A^_x = i k_y B^_z / k^2, A^_y = -i k_x B^_z / k^2; the mean and the
    Nyquist rows/columns are set to zero.  Returns [2, ny, nx]."""
    ny, nx = bz.shape
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=Lx / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=Ly / ny)
    KX, KY = np.meshgrid(kx, ky)
    k2 = KX ** 2 + KY ** 2
    k2[0, 0] = 1.0
    B = np.fft.fft2(bz)
    ax = 1j * KY * B / k2
    ay = -1j * KX * B / k2
    for a in (ax, ay):
        a[0, 0] = 0.0
        a[:, nx // 2] = 0.0
        a[ny // 2, :] = 0.0
    return np.stack([np.fft.ifft2(ax).real, np.fft.ifft2(ay).real])


# ---------------------------------------------------------------------------
# Step 1: ghost fill
# ---------------------------------------------------------------------------

def fill_ghosts(F, grid, par, lnrho0_z):
    """Fill every derived ghost cell of the ghosted state F in place.

    Periodic z: all faces periodic.  Solar z: the rules listed in the module
    docstring; the u_x, u_y values in the lower ghost planes are state and are
    left untouched.  z ghosts are set over the interior (x, y) first, then the
    x/y wrap runs over every plane so that edge and corner ghosts exist."""
    nz = grid["nz"]
    if grid["zbc"] == "periodic":
        F[:, :NG] = F[:, nz:nz + NG]
        F[:, nz + NG:] = F[:, NG:2 * NG]
        wrap_xy(F)
        return F
    z = zk(grid)
    ny, nx = grid["ny"], grid["nx"]
    kabs = _kabs_rfft(nx, ny, grid["Lx"], grid["Ly"])
    I = (slice(NG, NG + ny), slice(NG, NG + nx))
    k0, kt = NG, NG + nz - 1                   # array z-index of k = 0 and k = nz-1
    R, g = par["R"], par["g_z"]

    for c in (AX, AY, AZ):
        bot = F[c, k0][I].copy()
        top = F[c, kt][I].copy()
        for j in (1, 2, 3):
            # inverted potential field below (contrast grows with depth, reduced by f_bot)
            F[c, k0 - j][I] = kspace_filter(bot, np.exp(+par["f_bot"] * kabs * (z[k0] - z[k0 - j])))
            # potential field above, eq. (17)
            F[c, kt + j][I] = kspace_filter(top, np.exp(-kabs * (z[kt + j] - z[kt])))
    for j in (1, 2, 3):
        F[UZ, k0 - j][I] = -F[UZ, k0 + j][I]
        F[UZ, kt + j][I] = -F[UZ, kt - j][I]
        F[UX, kt + j][I] = F[UX, kt - j][I]
        F[UY, kt + j][I] = F[UY, kt - j][I]
        F[LNRHO, k0 - j][I] = lnrho0_z[k0 - j]
    # lower T: hydrostatic recursion, eq. (8):
    # ln p(-j) = ln p(-j+1) - (z(-j+1) - z(-j)) g/(R T(-j+1))
    for j in (1, 2, 3):
        up = k0 - j + 1
        F[LNT, k0 - j][I] = (F[LNT, up][I] + F[LNRHO, up][I] - F[LNRHO, k0 - j][I]
                             - (z[up] - z[k0 - j]) * g / (R * np.exp(F[LNT, up][I])))
    # upper T symmetric, eq. (11)
    for j in (1, 2, 3):
        F[LNT, kt + j][I] = F[LNT, kt - j][I]
    if not stretched(grid):
        # upper rho hydrostatic mirror, eq. (13) (symmetric grid distances)
        Ttop = np.exp(F[LNT, kt][I])
        for j in (1, 2, 3):
            F[LNRHO, kt + j][I] = F[LNRHO, kt - j][I] + g * (z[kt + j] - z[kt - j]) / (R * Ttop)
    else:
        # non-uniform z: the recursion of eq. (15), plane by plane upward
        for j in (1, 2, 3):
            Ta = np.exp(F[LNT, kt + j - 1][I])
            Tb = np.exp(F[LNT, kt + j][I])
            F[LNRHO, kt + j][I] = (F[LNRHO, kt + j - 1][I]
                                   + (z[kt + j] - z[kt + j - 1]) * 2.0 * g / (R * (Tb + Ta)))
    wrap_xy(F)
    return F


# ---------------------------------------------------------------------------
# radiation (continuous log-linear table) and its low-temperature cut
# ---------------------------------------------------------------------------

def ln_lambda(lnT, tab_lnT, tab_lnL):
    """Piecewise-linear ln Lambda~(ln T) through the breakpoints, constant
    outside the table.  The branch is chosen on the real part."""
    x = np.real(lnT)
    out = np.empty_like(lnT)
    n = len(tab_lnT)
    out[...] = tab_lnL[0]
    for i in range(n - 1):
        m = (x >= tab_lnT[i]) & (x < tab_lnT[i + 1])
        slope = (tab_lnL[i + 1] - tab_lnL[i]) / (tab_lnT[i + 1] - tab_lnT[i])
        out[m] = tab_lnL[i] + slope * (lnT[m] - tab_lnT[i])
    out[x >= tab_lnT[-1]] = tab_lnL[-1]
    return out


def rad_cut(lnT, lo, hi):
    """C^1 smoothstep in ln T from ln T_lo (0) to ln T_hi (1)."""
    a, b = math.log(lo), math.log(hi)
    s = (lnT - a) / (b - a)
    x = np.real(s)
    out = s * s * (3.0 - 2.0 * s)
    out = np.where(x <= 0.0, 0.0 * s, out)
    out = np.where(x >= 1.0, 1.0 + 0.0 * s, out)
    return out


def q_rad(rho, lnT, par):
    if len(par["rad_lnT"]) == 0:
        return 0.0 * rho
    return (rho * rho * np.exp(ln_lambda(lnT, par["rad_lnT"], par["rad_lnL"]))
            * rad_cut(lnT, par["T_rad_lo"], par["T_rad_hi"]))


def sine_cutoff(x, start, width):
    """1 for x <= start, 0 for x >= start + width, a sine transition between
    (1/2 [1 - sin(pi (x - start - width/2) / width)]).  Complex-safe: the
    branch is taken on the real part."""
    xr = np.real(x)
    mid = 0.5 * (1.0 - np.sin(np.pi * (x - start - 0.5 * width) / width))
    return np.where(xr <= start, 1.0, np.where(xr >= start + width, 0.0, mid))


def newton_cooling(lr, lT, z, k_index, par):
    """Chromospheric Newtonian cooling (Sect. 3.1, eqs. 9-10): contribution to
    d ln T/dt at zones with ln rho = lr, ln T = lT, height z (array index of
    the plane k_index, broadcast like lr).

    Target (eq. 9): T* = sqrt(T0(z) T'(rho)), T'(rho) = T0(z') at the height
    z' where the initial density equals the actual one, rho0(z') = rho.  The
    initial profiles are tabulated at the grid heights z_k, k = -3 .. nz+2
    (par['nc_lnrho0_z'], par['nc_lnT0_z']); z' is found by linear
    interpolation in ln rho0 between the bracketing nodes, clamped to the end
    values outside the table.
    Term (reading of the garbled eq. 10): d ln T/dt = -tau_t c_rho c_z (1 - T*/T),
    i.e. dT/dt = -tau_t c_rho c_z (T - T*), an exponential decay of T toward
    T* at the inverse time tau_t.
    Cutoffs: c_rho = 1 while ln rho is within nc_lnrho_magn - nc_lnrho_width
    natural-log orders of the photospheric density rho0(0), a sine down to 0
    over the last nc_lnrho_width orders; c_z = 1 below nc_z_max -
    nc_z_width, a sine down to 0 at nc_z_max."""
    tau = par.get("nc_tau", 0.0)
    if tau == 0.0:
        return 0.0 * lT
    x = np.asarray(par["nc_lnrho0_z"], dtype=np.float64)   # decreasing with z
    y = np.asarray(par["nc_lnT0_z"], dtype=np.float64)
    n = len(x)
    # bracketing segment [i, i+1] with x[i] >= lr > x[i+1], on the real part
    lrr = np.real(lr)
    i = np.sum(x[None, :] >= np.reshape(lrr, (-1, 1)), axis=1).reshape(np.shape(lrr)) - 1
    i = np.clip(i, 0, n - 2)
    w = (x[i] - lr) / (x[i] - x[i + 1])
    lTp = y[i] + w * (y[i + 1] - y[i])
    lTp = np.where(lrr >= x[0], y[0], np.where(lrr <= x[-1], y[-1], lTp))
    lTstar = 0.5 * (y[k_index] + lTp)
    c_rho = sine_cutoff(x[NG] - lr, par["nc_lnrho_magn"] - par["nc_lnrho_width"],
                        par["nc_lnrho_width"])
    c_z = sine_cutoff(z, par["nc_z_max"] - par["nc_z_width"], par["nc_z_width"])
    return -tau * c_rho * c_z * (1.0 - np.exp(lTstar - lT))


# ---------------------------------------------------------------------------
# Steps 2-3: right-hand side
# ---------------------------------------------------------------------------

def ramp(t, t_ramp):
    """Linear switch-on of the driver over t_ramp (Sect. 2.3)."""
    if t_ramp <= 0.0:
        return 1.0
    return min(1.0, t / t_ramp)


def driver_target(drv, t):
    """u* of eq. (5) at time t: the single target drv["uh"], or, for a pair of
    snapshots (drv["uh0"] at drv["t0"], drv["uh1"] at drv["t1"]), their linear
    interpolation in time with the weight clipped to [0, 1] (reading: the
    coronal run interpolates between granulation snapshots, Sect. 2.3)."""
    if "uh1" not in drv:
        return drv["uh"]
    w = min(1.0, max(0.0, (t - drv["t0"]) / (drv["t1"] - drv["t0"])))
    return drv["uh0"] + w * (drv["uh1"] - drv["uh0"])


def rhs(F, t, grid, par, drv):
    """Right-hand side at every interior zone, from a ghost-filled state F.

    Returns (R, Rg): R [8, nz, ny, nx] for the interior and Rg [2, 3, ny, nx]
    for u_x, u_y in the lower ghost planes k = -3, -2, -1 (solar only), which
    evolve under the nudging term of eq. (5) alone."""
    h = spacings(grid)
    nz = grid["nz"]
    solar = grid["zbc"] == "solar"
    gam, Rg_, mu0 = par["gamma"], par["R"], par["mu0"]
    eta, nu = par["eta"], par["nu"]
    cv = Rg_ / (gam - 1.0)

    val = [interior(F[c]) for c in range(8)]
    Ax, Ay, Az, ux, uy, uz, lr, lT = val
    u = (ux, uy, uz)
    A = (F[AX], F[AY], F[AZ])
    U = (F[UX], F[UY], F[UZ])

    # first derivatives GA[c][d] = d_d A_c, etc.
    GA = [[grad(A[c], d, h) for d in range(3)] for c in range(3)]
    Gu = [[grad(U[c], d, h) for d in range(3)] for c in range(3)]
    Gr = [grad(F[LNRHO], d, h) for d in range(3)]
    GT = [grad(F[LNT], d, h) for d in range(3)]

    # second derivatives; each mixed one computed once and used for both orders
    def full_hessian(f):
        H = [[None] * 3 for _ in range(3)]
        for i in range(3):
            for j in range(i, 3):
                H[i][j] = hess(f, i, j, h)
                H[j][i] = H[i][j]
        return H

    HA = [full_hessian(A[c]) for c in range(3)]
    Hu = [full_hessian(U[c]) for c in range(3)]
    HT = full_hessian(F[LNT])
    lap_r = sum(hess(F[LNRHO], d, d, h) for d in range(3))

    # magnetic field and its gradient, B = curl A (+ uniform external field)
    Bext = par["Bext"]
    B = (GA[2][1] - GA[1][2] + Bext[0],
         GA[0][2] - GA[2][0] + Bext[1],
         GA[1][0] - GA[0][1] + Bext[2])
    # dB[i][j] = d_j B_i
    dB = [[HA[2][j][1] - HA[1][j][2] for j in range(3)],
          [HA[0][j][2] - HA[2][j][0] for j in range(3)],
          [HA[1][j][0] - HA[0][j][1] for j in range(3)]]
    # mu0 J = curl B
    cB = (dB[2][1] - dB[1][2], dB[0][2] - dB[2][0], dB[1][0] - dB[0][1])

    rho = np.exp(lr)
    T = np.exp(lT)

    # swamp profile (solar only)
    z = zk(grid)[NG:NG + nz]
    if solar:
        w1, dw1 = swamp_weight(z, par["z_s"], par["z_t"])
    else:
        w1, dw1 = np.zeros(nz), np.zeros(nz)
    w = w1[:, None, None]
    dw = dw1[:, None, None]

    # --- induction equation (Weyl gauge, Sect. 2.4) + swamp eq. (18) -------
    uxB = (uy * B[2] - uz * B[1], uz * B[0] - ux * B[2], ux * B[1] - uy * B[0])
    divA = GA[0][0] + GA[1][1] + GA[2][2]
    RA = []
    for c in range(3):
        lapA = HA[c][0][0] + HA[c][1][1] + HA[c][2][2]
        r = uxB[c] - eta * cB[c] + par["eta_s"] * w * lapA
        if c == 2:
            r = r + par["eta_s"] * dw * divA
        RA.append(r)

    # --- momentum ---------------------------------------------------------
    divu = Gu[0][0] + Gu[1][1] + Gu[2][2]
    S = [[0.5 * (Gu[i][j] + Gu[j][i]) - (divu / 3.0 if i == j else 0.0) for j in range(3)]
         for i in range(3)]
    J = (cB[0] / mu0, cB[1] / mu0, cB[2] / mu0)
    JxB = (J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0])
    Ru = []
    for i in range(3):
        adv = u[0] * Gu[i][0] + u[1] * Gu[i][1] + u[2] * Gu[i][2]
        press = -Rg_ * T * (Gr[i] + GT[i])
        lap_u = Hu[i][0][0] + Hu[i][1][1] + Hu[i][2][2]
        graddiv = Hu[0][i][0] + Hu[1][i][1] + Hu[2][i][2]
        strain = S[i][0] * Gr[0] + S[i][1] * Gr[1] + S[i][2] * Gr[2]
        visc = nu * (lap_u + graddiv / 3.0 + 2.0 * strain)
        r = -adv + press + JxB[i] / rho + visc
        if i == 2:
            r = r + par["g_z"]
        Ru.append(r)

    # --- continuity (ln rho) with mass diffusion (Sect. 2.5) + swamp eq. (20)
    udr = u[0] * Gr[0] + u[1] * Gr[1] + u[2] * Gr[2]
    Rr = (-udr - divu + (par["D_rho"] + par["chi_rho"] * w) * lap_r
          + par["D_rho"] * (Gr[0] ** 2 + Gr[1] ** 2 + Gr[2] ** 2))

    # --- energy (ln T) --------------------------------------------------------
    ohm = eta * (cB[0] ** 2 + cB[1] ** 2 + cB[2] ** 2) / mu0
    SS = sum(S[i][j] * S[i][j] for i in range(3) for j in range(3))
    vheat = 2.0 * rho * nu * SS
    # field-aligned Spitzer conduction: div(kappa0 T^5/2 b (b.grad T)) expanded
    Bn = np.sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2] + par["B_floor"] ** 2)
    b = (B[0] / Bn, B[1] / Bn, B[2] / Bn)
    bG = b[0] * GT[0] + b[1] * GT[1] + b[2] * GT[2]
    bbH = sum(b[i] * b[j] * HT[i][j] for i in range(3) for j in range(3))
    v = [b[0] * dB[j][0] + b[1] * dB[j][1] + b[2] * dB[j][2] for j in range(3)]  # b_i d_i B_j
    vG = v[0] * GT[0] + v[1] * GT[1] + v[2] * GT[2]
    sbb = b[0] * v[0] + b[1] * v[1] + b[2] * v[2]
    Phi = par["kappa0"] * T ** 3.5
    qcond = Phi * (3.5 * bG * bG + bbH + (vG - 2.0 * bG * sbb) / Bn)
    qrad = q_rad(rho, lT, par)
    udT = u[0] * GT[0] + u[1] * GT[1] + u[2] * GT[2]
    lapT = HT[0][0] + HT[1][1] + HT[2][2]
    RT = (-udT - (gam - 1.0) * divu + (ohm + vheat + qcond - qrad) / (rho * cv * T)
          + par["chi_s"] * w * lapT)
    if par.get("nc_tau", 0.0) != 0.0:
        kk = np.arange(NG, NG + nz)[:, None, None] + np.zeros(lT.shape, dtype=int)
        zz = zk(grid)[kk]
        RT = RT + newton_cooling(lr, lT, zz, kk, par)

    R = np.stack(RA + Ru + [Rr, RT])
    Rgh = None
    if solar:
        s = ramp(t, par["t_ramp"])
        ustar, astar = driver_target(drv, t), drv["ah"]
        # nudging toward the driver, eq. (5), layers k = 0 .. -3
        for c in (0, 1):
            R[UX + c, 0] = R[UX + c, 0] - par["tau_u"] * (val[UX + c][0] - s * ustar[c])
            R[AX + c, 0] = R[AX + c, 0] - par["tau_A"] * (val[AX + c][0] - astar[c])
        Rgh = np.empty((2, NG) + ustar.shape[1:], dtype=R.dtype)
        for c in (0, 1):
            for j in range(NG):        # array z-index j = plane k = j - 3
                uh = F[UX + c, j, NG:-NG, NG:-NG]
                Rgh[c, j] = -par["tau_u"] * (uh - s * ustar[c])
        # closed boundaries: no RHS for u_z at both boundary planes, none for
        # ln rho at the photosphere (density held at the initial profile)
        R[UZ, 0] = 0.0
        R[UZ, nz - 1] = 0.0
        R[LNRHO, 0] = 0.0
    return R, Rgh


# ---------------------------------------------------------------------------
# Step 5: low-storage RK3 step
# ---------------------------------------------------------------------------

def rk3_step(F, t, dt, grid, par, lnrho0_z, drv=None):
    """One 2N-RK3 step (Williamson 1980).  F: ghosted state (not modified).
    Returns the new ghosted state (its derived ghosts are not refilled)."""
    F = F.copy()
    nz = grid["nz"]
    solar = grid["zbc"] == "solar"
    dF = np.zeros((8, nz, grid["ny"], grid["nx"]), dtype=F.dtype)
    dG = None
    for s in range(3):
        ts = t + RK_C[s] * dt
        fill_ghosts(F, grid, par, lnrho0_z)
        R, Rgh = rhs(F, ts, grid, par, drv)
        dF = RK_ALPHA[s] * dF + dt * R
        F[:, NG:NG + nz, NG:-NG, NG:-NG] += RK_BETA[s] * dF
        if solar:
            dG = Rgh * dt if dG is None else RK_ALPHA[s] * dG + dt * Rgh
            F[UX:UY + 1, 0:NG, NG:-NG, NG:-NG] += RK_BETA[s] * dG
            # re-impose the boundary values held by the closed/'fg' conditions
            F[UZ, NG, NG:-NG, NG:-NG] = 0.0
            F[UZ, NG + nz - 1, NG:-NG, NG:-NG] = 0.0
            F[LNRHO, NG, NG:-NG, NG:-NG] = lnrho0_z[NG]
        wrap_xy(F)
    return F


def run(F, t, dt, nsteps, grid, par, lnrho0_z, drv=None):
    for _ in range(nsteps):
        F = rk3_step(F, t, dt, grid, par, lnrho0_z, drv)
        t += dt
    return F, t


# ---------------------------------------------------------------------------
# Step 4: time step from the CFL and diffusion limits
# ---------------------------------------------------------------------------

def cfl_dt(F, grid, par):
    """dt = min(c_adv d/max(|u| + c_f), c_diff d^2/max D_eff,
    c_adv min(rho c_v T / Q_rad), c_nudge/max(tau_u, tau_A, tau_t)) over the
    interior, from a ghost-filled state F (reading: the paper gives only the
    Courant number 0.4 and the Spitzer limitation)."""
    h = spacings(grid)
    nz = grid["nz"]
    if stretched(grid):
        # reading: the z spacing of plane k is z'(k); delta per plane
        delta = np.minimum(min(h[0], h[1]), h[2].zp)[:, None, None]
    else:
        delta = min(h)
    gam, R, mu0 = par["gamma"], par["R"], par["mu0"]
    cv = R / (gam - 1.0)
    A = (F[AX], F[AY], F[AZ])
    GA = [[grad(A[c], d, h) for d in range(3)] for c in range(3)]
    Bext = par["Bext"]
    B = (GA[2][1] - GA[1][2] + Bext[0], GA[0][2] - GA[2][0] + Bext[1],
         GA[1][0] - GA[0][1] + Bext[2])
    ux, uy, uz = (interior(F[c]) for c in (UX, UY, UZ))
    rho = np.exp(interior(F[LNRHO]))
    lT = interior(F[LNT])
    T = np.exp(lT)
    B2 = B[0] ** 2 + B[1] ** 2 + B[2] ** 2
    cf = np.sqrt(gam * R * T + B2 / (mu0 * rho))
    speed = np.sqrt(ux ** 2 + uy ** 2 + uz ** 2) + cf
    if stretched(grid):
        dt = par["c_adv"] * np.min(delta / speed)
    else:
        dt = par["c_adv"] * delta / np.max(speed)

    z = zk(grid)[NG:NG + nz]
    if grid["zbc"] == "solar":
        w1, _ = swamp_weight(z, par["z_s"], par["z_t"])
    else:
        w1 = np.zeros(nz)
    w = w1[:, None, None] + 0.0 * rho
    D = np.maximum.reduce([
        par["nu"] + 0.0 * rho,
        par["eta"] + par["eta_s"] * w,
        par["D_rho"] + par["chi_rho"] * w,
        par["chi_s"] * w,
        par["kappa0"] * T ** 2.5 / (rho * cv),
    ])
    dmax = np.max(D)
    if dmax > 0 and stretched(grid):
        with np.errstate(divide="ignore"):
            dt = min(dt, par["c_diff"] * float(np.min(delta * delta / D)))
    elif dmax > 0:
        dt = min(dt, par["c_diff"] * delta * delta / dmax)
    qr = q_rad(rho, lT, par)
    if np.any(qr > 0):
        pos = qr > 0
        dt = min(dt, par["c_adv"] * np.min(rho[pos] * cv * T[pos] / qr[pos]))
    tau = max(par["tau_u"], par["tau_A"]) if grid["zbc"] == "solar" else 0.0
    tau = max(tau, par.get("nc_tau", 0.0))
    if tau > 0:
        dt = min(dt, par["c_nudge"] / tau)
    return float(dt)


# ---------------------------------------------------------------------------
# diagnostics used by the adjoint workload
# ---------------------------------------------------------------------------

def bz_at_height(F, grid, par, zq):
    """B_z = d_x A_y - d_y A_x (+ B_ext,z) on the horizontal plane at height
    zq, linear in z between the two enclosing grid planes."""
    h = spacings(grid)
    if stretched(grid):
        z = zk(grid)[NG:NG + grid["nz"]]
        k0 = min(int(np.searchsorted(z, zq, side="right")) - 1, grid["nz"] - 2)
        a = (zq - z[k0]) / (z[k0 + 1] - z[k0])
    else:
        kf = (zq - grid["z0"]) / h[2]
        k0 = int(math.floor(kf))
        a = kf - k0
    out = 0.0
    for k, wgt in ((k0, 1.0 - a), (k0 + 1, a)):
        if wgt == 0.0:
            continue
        Ay = F[AY, NG + k]                 # [ny+6, nx+6], x/y ghosts wrapped
        Ax = F[AX, NG + k]
        bz = d1(Ay, 1, h[0])[NG:-NG, :] - d1(Ax, 0, h[1])[:, NG:-NG]
        out = out + wgt * bz
    return out + par["Bext"][2]


def divergence_B(F, grid, par):
    """Discrete div B from the Hessian of A (each mixed term shared)."""
    h = spacings(grid)
    A = (F[AX], F[AY], F[AZ])
    HA = [[[hess(A[c], i, j, h) if i <= j else None for j in range(3)] for i in range(3)]
          for c in range(3)]

    def H(c, i, j):
        return HA[c][min(i, j)][max(i, j)]

    dBx_x = H(2, 0, 1) - H(1, 0, 2)
    dBy_y = H(0, 1, 2) - H(2, 1, 0)
    dBz_z = H(1, 2, 0) - H(0, 2, 1)
    return dBx_x + dBy_y + dBz_z


# ---------------------------------------------------------------------------
# tangent-linear reference by complex step (Squire & Trapp 1998)
# ---------------------------------------------------------------------------

def run_complex_step(F, dF, duh, t, dt, nsteps, grid, par, lnrho0_z, drv, h=1e-30):
    """Directional derivative of nsteps RK3 steps with respect to the state
    (direction dF, ghosted layout) and the driver target u* (direction duh):
    Im(step(F + i h dF; u* + i h duh)) / h.  Exact to round-off because every
    operation of the step is analytic in the perturbed quantities (branches
    are chosen on real parts).  Returns (value, derivative), both ghosted."""
    Fc = F.astype(complex) + 1j * h * dF
    drvc = None
    if drv is not None:
        uh = drv["uh"].astype(complex)
        if duh is not None:
            uh = uh + 1j * h * duh
        drvc = dict(uh=uh, ah=drv["ah"])
    out, _ = run(Fc, t, dt, nsteps, grid, par, lnrho0_z, drvc)
    return out.real, out.imag / h


def bz_misfit_loss(F, grid, par, zq, target):
    """L = 1/2 sum_xy (B_z(x, y, zq) - target)^2."""
    d = bz_at_height(F, grid, par, zq) - target
    return 0.5 * np.sum(d * d)
