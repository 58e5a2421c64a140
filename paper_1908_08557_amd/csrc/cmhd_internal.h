// Internal declarations of the gfx950 MHD library that the kernels are built
// from: kernel parameter block, field indices, tile geometry and device
// helpers.  The host-side launch helpers are declared in launch.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cmhd.h"

namespace cmhd {

constexpr int NG = 3;   // ghost planes per side (three ghost layers, Sect. 2.3-4.2)
constexpr int NF = 8;   // Ax Ay Az ux uy uz lnrho lnT
enum Field { AX = 0, AY, AZ, UX, UY, UZ, LR, LT };

// Tile of the fused stencil kernel: 16 x 16 columns, one thread per column,
// marching in z; the x/y halo of 3 points makes a 22 x 22 plane in LDS.
constexpr int TX = 16, TY = 16, NT = TX * TY;
constexpr int HX = TX + 2 * NG, HY = TY + 2 * NG, HP = HX * HY;
constexpr int NHALO = HP - NT;   // 228 halo points per plane

// Parameter block handed to every kernel by value.
struct KParams {
  int nx, ny, nz, solar;
  long long splane;   // nx*ny: z stride
  long long sfield;   // (nz+6)*nx*ny: field stride
  double dx, dy, dz, z0;
  double i60dx, i60dy, i60dz;      // 1/(60 h)
  double i180dx2, i180dy2, i180dz2;  // 1/(180 h^2)
  double gamma, R, mu0, inv_mu0, eta, nu, D_rho, kappa0, g_z, cv, inv_cv, gm1;
  double Bext[3];
  double B_floor2;
  double eta_s, chi_s, chi_rho, z_s, z_t;
  double tau_u, tau_A, f_bot;
  int n_rad;
  double rad_lnT[CMHD_MAX_RAD], rad_lnL[CMHD_MAX_RAD], rad_slope[CMHD_MAX_RAD];
  double lnT_rad_lo, lnT_rad_hi, inv_dlnT_rad;
  double lnrho0_bot[4];   // ln rho0 at k = -3, -2, -1, 0
  double Lx, Ly;
  double c_adv, c_diff, c_nudge;
  // chromospheric Newtonian cooling: rate, start and width of the density
  // cutoff (in natural-log orders below ln rho0 at z0), of the height cutoff,
  // the photospheric ln rho0, the ends and middles of the two cutoffs and
  // pi over their widths, the table length (nz+6) and the device copy of
  // the initial profiles [ln rho0 (nc_n) | ln T0 (nc_n)]
  double nc_tau, nc_dlr0, nc_dlrw, nc_z0, nc_zw, nc_lnrho_phot;
  double nc_dlr1, nc_dlrm, nc_z1, nc_zm, nc_pi_dlrw, nc_pi_zw;
  int nc_n;
  const double* nc_tab;
  // non-uniform z grid (stretched != 0; uniform grids use z0 + k dz):
  // spacings of the ghost planes, the distances of the potential-field
  // filters, min(dx, dy), and the device table ztab = [z_k (nz+6) |
  // c1 = 1/(60 z') | c2 = 1/(180 z'^2) | c3 = -z''/(60 z'^3) | z' (nz each)]
  int stretched;
  double dz_lo[3];       // z(-j+1) - z(-j), j = 1..3
  double dz_hi[3];       // z(nz-1+j) - z(nz-2+j), j = 1..3
  double pf_dist[2][3];  // below: -f_bot (z(0) - z(-j)); above: z(nz-1+j) - z(nz-1)
  double dxy_min;
  const double* ztab;
};

// offsets in KParams::ztab
__host__ __device__ inline int zt_c1(const KParams& p) { return p.nz + 6; }
__host__ __device__ inline int zt_c2(const KParams& p) { return 2 * p.nz + 6; }
__host__ __device__ inline int zt_c3(const KParams& p) { return 3 * p.nz + 6; }
__host__ __device__ inline int zt_zp(const KParams& p) { return 4 * p.nz + 6; }
__host__ __device__ inline int zt_size(const KParams& p) { return 5 * p.nz + 6; }

// height of plane k (k = -3 .. nz+2; k uniform across the wave).  The table
// is read through the constant address space: a scalar load, which the
// kernels' in-flight global->LDS copies do not hold up (a vector load here
// would make the plane loop wait for them)
__device__ __forceinline__ double zk(const KParams& p, int k) {
  if (!p.stretched) return p.z0 + k * p.dz;
  const __attribute__((address_space(4))) double* t =
      (const __attribute__((address_space(4))) double*)p.ztab;
  return t[k + 3];
}

// Per-substage arguments of the Runge-Kutta update.
struct StageArgs {
  double alpha, beta, dt, ramp;
};

// Williamson (1980) 2N-storage RK3.
constexpr double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
constexpr double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
constexpr double RK_C[3] = {0.0, 1.0 / 3.0, 3.0 / 4.0};

// |k| of the Fourier mode at index (ix, iy) (FFT order, Nyquist at -n/2)
__device__ __forceinline__ double kabs(const KParams& p, int ix, int iy) {
  const int mx = ix < p.nx / 2 ? ix : ix - p.nx;
  const int my = iy < p.ny / 2 ? iy : iy - p.ny;
  const double kx = 6.283185307179586476925286766559 * mx / p.Lx;
  const double ky = 6.283185307179586476925286766559 * my / p.Ly;
  return sqrt(kx * kx + ky * ky);
}

// Scratch of the Fourier boundary: complex planes needed by
// launch_potential_ghosts (4 forward + 12 filtered).
constexpr int FFT_PLANES = 16;

__host__ __device__ inline int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

}  // namespace cmhd
