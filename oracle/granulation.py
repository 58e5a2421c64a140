"""Plain FP64 CPU oracle of the photospheric granulation driver (Sect. 2.3,
"Granulation driver", eqs. 1-4) and of the linear time interpolation between
two driver snapshots that the coronal model nudges toward (Sect. 2.3, the
two-step scheme).

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or calls
this file; only the test suite, the smoke check and the CPU baseline of the
benchmark do.  It shares no code with the library.

Random numbers are inputs: the caller passes a pool of uniforms in [0, 1)
(one per birth, for the birth position) and a pool of variations in [-1, 1]
(two per birth: lifetime and amplitude); a fill that needs more than the pool
holds raises PoolExhausted.

What the paper fixes:
  * granules of 1.6 Mm diameter (radius r_gran = 0.8 Mm) with a further
    0.24 Mm around each in which inter-granular lanes form by overlap, so a
    granule's field reaches r_lane = 1.04 Mm; the radial speed is zero at the
    centre, grows outward, and decays between 0.8 and 1.04 Mm;
  * the domain is filled at random until no space is left; no granule is
    born closer than r_excl = 0.64 Mm to a living centre;
  * lifetime T = T_gran (5 min) and amplitude v_max = v0 (1.028 km/s) varied
    per granule by normally distributed amounts within 10 % and 15 %;
  * t_max = T sqrt(|ln(v_min / v_max)|) (eq. 1) and the life cycle
    v(t) = v_max exp(-((t - t0 - t_max) / T)^2) (eq. 2), v_min = 0.78 v0; a
    granule ceases to exist once v(t) < v_min and its area is free again;
  * the rotational part of the 2-D field is filtered with
    exp(-(2 |k| / k_N)^4) (eq. 3), amplified by f_rot = 5 and added back, and
    the sum is rescaled to the rms of the granular field (eq. 4);
  * granule centres move with an external velocity field when one is given
    and stay put otherwise.
Readings (the paper gives the above in words only):
  1. Velocity of one granule: v(t) g(r) r_hat with g = r / r_gran for
     r < r_gran, g = (1 + cos(pi (r - r_gran) / (r_lane - r_gran))) / 2 for
     r_gran <= r < r_lane, g = 0 beyond (continuous, one at r_gran); the
     fields of all granules are summed (overlaps give the non-radial lanes),
     with the nearest periodic image of every centre.
  2. Filling is random sequential addition on the pixel lattice: a pixel
     (x_i = i dx, y_j = j dy) is free when every living centre lies at least
     r_excl away (squared distances compared); each birth takes the
     floor(u n)-th free pixel in raster order (y slowest) for the next
     uniform u, n the number of free pixels, until none is free.  A newborn
     granule starts at t0 = the update time.
  3. "Within 10 %" / "within 15 %": T = T_gran (1 + 0.10 xi_T),
     v_max = v0 (1 + 0.15 xi_v) with xi drawn from the standard normal
     truncated to [-1, 1] (so v_max > v_min always).
  4. Death is tested at update times, as t > t0 + 2 t_max, which is v(t) <
     v_min for t >= t0 (eq. 2) without rounding at the birth instant.
  5. Advection of the centres (external field given): forward Euler over the
     time since the previous update, velocity bilinear in the periodic
     pixel grid at the centre, position wrapped into [0, L).
  6. Eq. (3): rotational part = the divergence-free (Helmholtz) projection
     v^ - k (k . v^) / |k|^2, zero at k = 0 and on the Nyquist row and column
     (there the sign of the wave vector is undefined and the projection of a
     real field would not stay real; the filter is exp(-16) there anyway);
     k_N = pi / max(dx, dy).
The linear time interpolation between two snapshots (the nudging target of
the coronal run) is mhd.driver_target.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(
    r_gran=0.8,          # Mm
    r_lane=1.04,         # Mm
    r_excl=0.64,         # Mm
    t_gran=0.3,          # ks (5 min)
    v0=1.028,            # km/s
    vmin_frac=0.78,
    life_var=0.10,
    amp_var=0.15,
    f_rot=5.0,
)


class PoolExhausted(RuntimeError):
    pass


def params(nx, ny, Lx, Ly, **over):
    p = dict(DEFAULTS)
    p.update(nx=nx, ny=ny, Lx=Lx, Ly=Ly)
    p.update(over)
    return p


# ---------------------------------------------------------------------------
# life cycle, eqs. (1)-(2)
# ---------------------------------------------------------------------------

def t_max(T, vmax, vmin):
    """Eq. (1)."""
    return T * math.sqrt(abs(math.log(vmin / vmax)))


def amplitude(t, t0, T, vmax, tmax):
    """Eq. (2)."""
    a = (t - t0 - tmax) / T
    return vmax * math.exp(-(a * a))


def is_dead(t, t0, tmax):
    """Reading 4: v(t) < v_min for t >= t0."""
    return t > t0 + 2.0 * tmax


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def periodic_delta(d, L):
    """Nearest periodic image of a separation d (arrays or scalars)."""
    return d - L * np.floor(d / L + 0.5)


def wrap(x, L):
    return x - L * math.floor(x / L)


def profile(r, p):
    """Reading 1: g(r)."""
    rg, rl = p["r_gran"], p["r_lane"]
    inner = r / rg
    lane = 0.5 * (1.0 + np.cos(np.pi * (r - rg) / (rl - rg)))
    return np.where(r < rg, inner, np.where(r < rl, lane, 0.0))


def pixel_coords(p):
    dx, dy = p["Lx"] / p["nx"], p["Ly"] / p["ny"]
    return np.arange(p["nx"]) * dx, np.arange(p["ny"]) * dy


# ---------------------------------------------------------------------------
# the granule population
# ---------------------------------------------------------------------------

class Granules:
    """Living granules: centre (x, y), birth time t0, lifetime T, amplitude
    v_max and time of maximum t_max, in birth order."""

    def __init__(self):
        self.g = []          # rows [x, y, t0, T, vmax, tmax]

    def array(self):
        return np.array(self.g, dtype=float).reshape(-1, 6)

    def __len__(self):
        return len(self.g)


def free_mask(gr, p):
    """Reading 2: pixel free when every living centre is >= r_excl away."""
    X, Y = pixel_coords(p)
    r2 = p["r_excl"] * p["r_excl"]
    free = np.ones((p["ny"], p["nx"]), dtype=bool)
    for x, y, *_ in gr.g:
        dx = periodic_delta(X - x, p["Lx"])
        dy = periodic_delta(Y - y, p["Ly"])
        d2 = dy[:, None] * dy[:, None] + dx[None, :] * dx[None, :]
        free &= ~(d2 < r2)
    return free


def fill(gr, t, p, unif, xi, cursor):
    """Random sequential addition until no pixel is free (reading 2).
    Consumes unif[cursor], xi[2 cursor], xi[2 cursor + 1] per birth and
    returns the new cursor."""
    X, Y = pixel_coords(p)
    nx = p["nx"]
    r2 = p["r_excl"] * p["r_excl"]
    vmin = p["vmin_frac"] * p["v0"]
    free = free_mask(gr, p)
    while True:
        idx = np.flatnonzero(free.ravel())
        n = idx.size
        if n == 0:
            return cursor
        if cursor >= len(unif) or 2 * cursor + 1 >= len(xi):
            raise PoolExhausted(f"birth {cursor}: random pool exhausted")
        k = min(int(math.floor(unif[cursor] * n)), n - 1)
        iy, ix = divmod(int(idx[k]), nx)
        xc, yc = X[ix], Y[iy]
        T = p["t_gran"] * (1.0 + p["life_var"] * xi[2 * cursor])
        vmax = p["v0"] * (1.0 + p["amp_var"] * xi[2 * cursor + 1])
        gr.g.append([xc, yc, t, T, vmax, t_max(T, vmax, vmin)])
        cursor += 1
        dx = periodic_delta(X - xc, p["Lx"])
        dy = periodic_delta(Y - yc, p["Ly"])
        d2 = dy[:, None] * dy[:, None] + dx[None, :] * dx[None, :]
        free &= ~(d2 < r2)


def sample_bilinear(v, x, y, p):
    """Periodic bilinear sample of the plane v [ny][nx] at (x, y)."""
    nx, ny = p["nx"], p["ny"]
    fx = x / (p["Lx"] / nx)
    fy = y / (p["Ly"] / ny)
    i0, j0 = math.floor(fx), math.floor(fy)
    a, b = fx - i0, fy - j0
    i0, j0 = i0 % nx, j0 % ny
    i1, j1 = (i0 + 1) % nx, (j0 + 1) % ny
    return ((1.0 - a) * (1.0 - b) * v[j0, i0] + a * (1.0 - b) * v[j0, i1]
            + (1.0 - a) * b * v[j1, i0] + a * b * v[j1, i1])


class Driver:
    """The 2-D granulation run: a granule population advanced from update to
    update, and the velocity field it drives."""

    def __init__(self, p):
        self.p = p
        self.gr = Granules()
        self.t_last = None
        self.cursor = 0

    def update(self, t, unif, xi, vext=None):
        """Advance the population to time t: advect the centres (reading 5),
        remove dead granules (reading 4), refill (reading 2).  Returns the
        number of births."""
        p = self.p
        if vext is not None and self.t_last is not None:
            h = t - self.t_last
            for g in self.gr.g:
                ux = sample_bilinear(vext[0], g[0], g[1], p)
                uy = sample_bilinear(vext[1], g[0], g[1], p)
                g[0] = wrap(g[0] + ux * h, p["Lx"])
                g[1] = wrap(g[1] + uy * h, p["Ly"])
        self.gr.g = [g for g in self.gr.g if not is_dead(t, g[2], g[5])]
        c0 = self.cursor
        self.cursor = fill(self.gr, t, p, unif, xi, self.cursor)
        self.t_last = t
        return self.cursor - c0

    def velocity(self, t):
        """Driver velocity at time t: granular field, eqs. (3)-(4)."""
        return enhance_vorticity(granular_field(self.gr, t, self.p), self.p)


# ---------------------------------------------------------------------------
# the velocity field
# ---------------------------------------------------------------------------

def granular_field(gr, t, p):
    """v_gran(r, t): the summed fields of all granules (reading 1).
    Returns [2, ny, nx]."""
    X, Y = pixel_coords(p)
    v = np.zeros((2, p["ny"], p["nx"]))
    for x, y, t0, T, vmax, tm in gr.g:
        a = amplitude(t, t0, T, vmax, tm)
        dx = periodic_delta(X - x, p["Lx"])[None, :]
        dy = periodic_delta(Y - y, p["Ly"])[:, None]
        r = np.sqrt(dx * dx + dy * dy)
        rs = np.where(r > 0.0, r, 1.0)
        s = np.where(r > 0.0, a * profile(r, p) / rs, 0.0)
        v[0] += s * dx
        v[1] += s * dy
    return v


def rotational_part(v, p):
    """Divergence-free projection of a periodic 2-D field, filtered with
    eq. (3) (reading 6).  Returns [2, ny, nx]."""
    nx, ny = p["nx"], p["ny"]
    dx, dy = p["Lx"] / nx, p["Ly"] / ny
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dy)
    KX, KY = np.meshgrid(kx, ky)
    k2 = KX * KX + KY * KY
    k2s = np.where(k2 > 0.0, k2, 1.0)
    Vx, Vy = np.fft.fft2(v[0]), np.fft.fft2(v[1])
    proj = (KX * Vx + KY * Vy) / k2s
    Wx, Wy = Vx - KX * proj, Vy - KY * proj
    for W_ in (Wx, Wy):
        W_[0, 0] = 0.0
        W_[:, nx // 2] = 0.0
        W_[ny // 2, :] = 0.0
    kN = np.pi / max(dx, dy)
    filt = np.exp(-(2.0 * np.sqrt(k2) / kN) ** 4)
    return np.stack([np.fft.ifft2(Wx * filt).real, np.fft.ifft2(Wy * filt).real])


def enhance_vorticity(v, p):
    """Eqs. (3)-(4): v_vor = v + f_rot v_rot', rescaled to the rms of v."""
    vvor = v + p["f_rot"] * rotational_part(v, p)
    num = np.mean(v[0] * v[0] + v[1] * v[1])
    den = np.mean(vvor[0] * vvor[0] + vvor[1] * vvor[1])
    if den == 0.0:
        return np.zeros_like(v)
    return vvor * math.sqrt(num / den)
