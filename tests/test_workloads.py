"""The seeded input generators against the properties the input recipe
states: balanced, Nyquist-free bipoles with the requested peak; an initial
A_h whose curl is that B_z and whose modes decay as exp(-|k| z); a
divergence-free driver of the requested rms; a hydrostatic ln rho0 exact for
a constant temperature; monotone stretched heights; truncated normal pools.
Checks are spectral (numpy FFTs) or closed forms, independent of the
generators' own construction order."""
import math

import numpy as np

from paper_1908_08557_amd import workloads as W


def _k(nx, ny, L):
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=L / nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=L / ny)
    return np.meshgrid(kx, ky)


def test_bipoles_balanced_nyquist_free_and_peaked():
    bz = W.bipole_field(64, 32, 20.0, 20.0, 3, 7, 1.5, 2.0, 6.0)
    assert bz.shape == (32, 64)
    assert abs(bz.mean()) < 1e-14 * np.abs(bz).max()
    assert np.abs(bz).max() == 1.5
    B = np.fft.fft2(bz)
    assert np.abs(B[:, 32]).max() < 1e-12 * np.abs(B).max()
    assert np.abs(B[16, :]).max() < 1e-12 * np.abs(B).max()
    assert np.array_equal(bz, W.bipole_field(64, 32, 20.0, 20.0, 3, 7, 1.5, 2.0, 6.0))


def test_potential_A_curl_and_decay():
    L, n = 16.0, 32
    bz = W.bipole_field(n, n, L, L, 2, 4, 1.0, 1.5, 4.0)
    z = np.array([0.0, 0.7])
    A = W.potential_A_from_bz(bz, L, L, z)
    KX, KY = _k(n, n, L)
    K = np.sqrt(KX ** 2 + KY ** 2)
    for i, zz in enumerate(z):
        curl = np.real(np.fft.ifft2(1j * KX * np.fft.fft2(A[1, i]) - 1j * KY * np.fft.fft2(A[0, i])))
        expect = np.real(np.fft.ifft2(np.fft.fft2(bz) * np.exp(-K * zz)))
        assert np.abs(curl - expect).max() < 1e-12 * np.abs(bz).max()


def test_driver_divergence_free_with_rms():
    u = W.solenoidal_uh(48, 32, 12.0, 12.0, seed=5, rms=1.0, ell=1.0)
    KX, KY = np.meshgrid(2 * np.pi * np.fft.fftfreq(48, d=12.0 / 48),
                         2 * np.pi * np.fft.fftfreq(32, d=12.0 / 32))
    div = np.real(np.fft.ifft2(1j * KX * np.fft.fft2(u[0]) + 1j * KY * np.fft.fft2(u[1])))
    assert np.abs(div).max() < 1e-12 * np.abs(u).max()
    assert abs(math.sqrt(np.mean(u[0] ** 2 + u[1] ** 2)) - 1.0) < 1e-14


def test_hydrostatic_profile_exact_for_constant_temperature():
    R, g, T = 0.01376, -274.0, 8.0e3
    z = np.linspace(-1.5, 6.0, 16)
    z = z - z[np.argmin(np.abs(z))]            # a plane at z = 0
    lnr = W.hydrostatic_lnrho(z, lambda s: np.full_like(np.asarray(s, dtype=float), T), R, g, 2.7)
    assert np.allclose(lnr, math.log(2.7) + g * z / (R * T), rtol=0, atol=1e-12)


def test_stretched_heights_monotone_between_spacings():
    z = W.stretched_heights(64, 0.0, 0.1, 0.8, 20.0, 6.0)
    dz = np.diff(z)
    assert len(z) == 64 + 6 and np.all(dz > 0)
    assert abs(z[3]) < 1e-12                    # plane k = 0 at z0
    assert 0.1 - 1e-3 < dz.min() and dz.max() < 0.8 + 1e-3
    assert dz[0] < 0.11 and dz[-1] > 0.79


def test_granulation_pools():
    u, xi = W.granulation_randoms(5000, 3)
    assert u.shape == (5000,) and xi.shape == (10000,)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert np.abs(xi).max() <= 1.0
    assert abs(xi.mean()) < 0.05 and 0.2 < xi.std() < 0.6   # a unit normal truncated at 1
