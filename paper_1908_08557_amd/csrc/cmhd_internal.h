// Internal declarations of the gfx950 MHD library: kernel parameter block,
// field indices, tile geometry and the launch helpers shared by the
// translation units.
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
  double gamma, R, mu0, inv_mu0, eta, nu, D_rho, kappa0, g_z, cv, gm1;
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
  // the photospheric ln rho0, the table length (nz+6) and the device copy of
  // the initial profiles [ln rho0 (nc_n) | ln T0 (nc_n)]
  double nc_tau, nc_dlr0, nc_dlrw, nc_z0, nc_zw, nc_lnrho_phot;
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

// Launchers (each returns the hipError_t of its launch).
// bytes of the z-derivative buffer (16 slots of nz planes, in the precision
// of the right-hand side)
size_t zderiv_bytes(const KParams& p, int prec);
// How a substage is cut into z chunks: the fused kernel marches kchunk planes
// per block.  pipelined: one fused launch per chunk, the z-derivative pass of
// chunk c overlapping the fused kernel of chunk c-1 on a second stream.
struct ChunkPlan {
  int kchunk, nchunk;
  bool pipelined;
};
ChunkPlan plan_chunks(const KParams& p);
// z derivatives of planes [k0, k1)
hipError_t launch_zderiv(const KParams& p, int prec, const double* f, void* dz, int k0, int k1,
                         hipStream_t s);
// fused substage kernel over the chunks [chunk0, chunk0 + nchunks) of the plan
hipError_t launch_rhs_rk(const KParams& p, int prec, int stage, const double* f, const void* dz,
                         double* fo, double* dF, const double* uh, const double* ah,
                         StageArgs st, const ChunkPlan& cp, int chunk0, int nchunks,
                         hipStream_t s);
hipError_t launch_ghost_rows(const KParams& p, const double* f, double* fo, double* dF,
                             const double* uh, StageArgs st, int read_dF, int write_dF,
                             hipStream_t s);
hipError_t launch_fill_periodic_z(const KParams& p, double* f, hipStream_t s);
// B_z on the plane (1 - a) z_k0 + a z_k0+1 (any grid)
hipError_t launch_bz_plane_k(const KParams& p, const double* f, int k0, double a, double* dst,
                             hipStream_t s);
hipError_t launch_fill_solar_columns(const KParams& p, double* f, hipStream_t s);
hipError_t launch_potential_ghosts(const KParams& p, double* f, double2* scratch,
                                   hipStream_t s);
hipError_t launch_ah_from_bz(const KParams& p, const double* bz, double* ah, double2* scratch,
                             hipStream_t s);
hipError_t launch_cfl_max(const KParams& p, const double* f, unsigned long long* out3,
                          hipStream_t s);
hipError_t launch_bz_plane(const KParams& p, const double* f, double zq, double* dst,
                           hipStream_t s);
hipError_t launch_finite_check(const KParams& p, const double* f, int* flag, hipStream_t s);
hipError_t launch_sum_abs(const KParams& p, const double* plane, double* out2, hipStream_t s);

// tangent-linear and adjoint pieces (adjoint.hip); Q holds the 72 pointwise
// inputs of every interior zone, [72][nz*ny*nx]
constexpr int NQ_POINT = 72;
hipError_t launch_point_q(const KParams& p, const double* g, double* Q, hipStream_t s);
hipError_t launch_point_jvp(const KParams& p, const double* Q, const double* dQ, const double* uh,
                            const double* ah, const double* duh, double ramp, double* dR,
                            hipStream_t s);
hipError_t launch_ghost_rows_jvp(const KParams& p, const double* dX, const double* duh,
                                 double ramp, double* dR, hipStream_t s);
hipError_t launch_point_vjp(const KParams& p, const double* Q, const double* Rbar,
                            const double* uh, const double* ah, double ramp, double* Qbar,
                            double* uhbar, hipStream_t s);
hipError_t launch_ghost_rows_vjp(const KParams& p, const double* Rbar, double ramp, double* Xbar,
                                 double* uhbar, hipStream_t s);
hipError_t launch_stencil_T(const KParams& p, const double* Qbar, double* Gbar, hipStream_t s);
hipError_t launch_fill_lin(const KParams& p, const double* g, double* dg, double2* scratch,
                           hipStream_t s);
hipError_t launch_fold_ghosts_T(const KParams& p, const double* g, const double* Gbar,
                                double* Xbar, double2* scratch, hipStream_t s);
hipError_t launch_tlm_combine(const KParams& p, double alpha, double beta, double dt,
                              const double* dR, double* dDF, double* dX, hipStream_t s);
hipError_t launch_adj_combine(const KParams& p, double alpha, double beta, double dt, double* Xb,
                              double* dFb, double* Rb, hipStream_t s);
hipError_t launch_copy_state_entries(const KParams& p, const double* src, double* dst,
                                     hipStream_t s);
hipError_t launch_bz_plane_vjp(const KParams& p, double zq, const double* bzbar, double* Xbar,
                               hipStream_t s);
hipError_t launch_bz_plane_vjp_k(const KParams& p, int k0, double a, const double* bzbar,
                                 double* Xbar, hipStream_t s);

// uh = u0 + w (u1 - u0) over the two driver planes [2][ny][nx]
hipError_t launch_driver_interp(const KParams& p, const double* u0, const double* u1, double w,
                                double* uh, hipStream_t s);

// 2-D FFT of nplanes complex planes [ny][nx] in place: sign -1 forward
// (unnormalised), +1 inverse (unnormalised; the filters carry 1/(nx ny)).
hipError_t fft2d(const KParams& p, double2* d, int nplanes, double sign, hipStream_t s);

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
