// Host-side launch helpers shared by the translation units of the library
// (each returns the hipError_t of its launch).  Declarations only: the
// kernels themselves are built from cmhd_internal.h and their own sources.
#pragma once

#include "cmhd_internal.h"

namespace cmhd {

// How a substage is cut into z chunks: each block of the fused substage
// kernel marches kchunk planes of one 16 x 16 tile.
struct SubstagePlan {
  int kchunk, nchunk;
};
SubstagePlan plan_substage(const KParams& p);
// one substage from f to fo: stencils, right-hand side and 2N-RK3 update of
// every interior zone (ghosts of f filled); pg: a device copy of p
hipError_t launch_substage(const KParams& p, const KParams* pg, int prec, int stage,
                           const double* f, double* fo, double* dF, const double* uh,
                           const double* ah, StageArgs st, hipStream_t s);
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

}  // namespace cmhd
