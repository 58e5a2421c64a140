// Pointwise right-hand side of the MHD system at one zone.  The zone's
// values and first/second derivatives are pulled on demand from a source
// object, in an order that keeps few values alive: first the magnetic field
// and its gradient, then the velocity gradient, then ln rho and ln T.
//
// Templated on the scalar type S: double (FP64 path), float (split path:
// derivatives arrive in float; the conduction coefficient, rho, T and the
// radiative-loss exponent are formed in double from the double state) and the
// forward-mode dual numbers of the tangent and adjoint kernels.
//
// Equations (the paper prints only its added terms, Sects. 2-4):
//   dA/dt   = u x B - eta mu0 J + eta_s w lap A + e_z eta_s w' div A     (eq. 18)
//             - tau_A (A_h - A_h*)                          photosphere only
//   du/dt   = -(u.grad)u - R T grad(ln rho + ln T) + J x B / rho + g e_z
//             + nu (lap u + grad div u / 3 + 2 S.grad ln rho)
//             - tau_u (u_h - s(t) u*)                          photosphere (eq. 5)
//   dlnrho  = -u.grad ln rho - div u + (D_rho + chi_rho w) lap ln rho
//             + D_rho |grad ln rho|^2                          (Sect. 2.5, eq. 20)
//   dlnT    = -u.grad ln T - (gamma-1) div u + chi_s w lap ln T         (eq. 19)
//             + [eta mu0 J^2 + 2 rho nu S:S + Q_cond - Q_rad] / (rho c_v T)
// with B = curl A + B_ext (eqs. 6-7), mu0 J = curl B, S the traceless rate of
// strain, Q_cond = div(kappa0 T^5/2 b b.grad T) (Spitzer) expanded with
// div B = 0 into
//   kappa0 T^7/2 [7/2 (b.G)^2 + b b:H + (b_i d_i B_j G_j - 2 (b.G) b_i b_k d_i B_k)/|B|_r]
// (G, H gradient and Hessian of ln T, b = B/|B|_r), and Q_rad = rho^2 Lambda(T) W(T).
//
// Source interface (f a field index, slot a Hessian slot xx yy zz xy xz yz):
//   S v(f); double v64(f); S d(f, dir); S lapr();
//   void grad(f, S g[3]): the gradient of f;
//   void gh(f, S g[3], S h[6]): gradient and Hessian of f together (only the
//   Hessian slots the equations use need be filled);
//   kUnrollA, kUnrollU: unroll factors of the component loops over A and u
//   (1 keeps a source's on-demand reads in a rolled loop).
//
// The evaluation is split into pieces that a kernel may run on different
// waves: the magnetic part (induction, B, J, the Spitzer field direction),
// the terms it hands to the fluid equations (Lorentz force, Ohmic and
// conductive heating, the swamp diffusion of ln T), the rest of the fluid
// equations, and the boundary terms; rhs_eval runs them all.
#pragma once

#include <type_traits>

#include "cmhd_internal.h"

namespace cmhd {

// Hessian slot of d_i d_j: xx, yy, zz, xy, xz, yz
__host__ __device__ constexpr int hslot(int i, int j) {
  return i == j ? i : (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5));
}

template <typename S>
struct PointCtx {
  double w, dw;       // swamp weight and its z-derivative at this plane
  int bottom, top;    // photospheric / top boundary plane (solar mode)
  S uh[2];            // driver u* at (x, y)
  S ah[2];            // A_h* at (x, y)
  double ramp;        // s(t)
  double nc_cz;       // height cutoff c_z of the Newtonian cooling at this plane
  double nc_lnT0;     // ln T0 at this plane's height (its reference profile)
};

// math helpers overloaded on the scalar type
__device__ inline double s_exp(double a) { return exp(a); }
__device__ inline float s_exp(float a) { return expf(a); }
__device__ inline double s_sqrt(double a) { return sqrt(a); }
__device__ inline float s_sqrt(float a) { return __fsqrt_rn(a); }
// 1/sqrt(a), a > 0: the hardware estimate refined by two Newton-Raphson
// steps y <- y + y (1 - a y^2) / 2 (each at least doubles the correct bits;
// the result is within a few units in the last place, not correctly rounded)
__device__ inline double s_rsqrt(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double e = fma(-a * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-a * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ inline float s_rsqrt(float a) { return 1.0f / __fsqrt_rn(a); }
__device__ inline double s_sin(double a) { return sin(a); }
__device__ inline double value_of(double a) { return a; }

// 1 for x <= start, 0 for x >= end = start + width, 1/2 [1 - sin(pi (x -
// mid) / width)] between, mid = start + width/2 (the sine cutoffs of the
// Newtonian cooling); end, mid and pi_w = pi / width are formed on the host
template <typename S>
__device__ inline S sine_cutoff(S x, double start, double end, double mid, double pi_w) {
  const double xv = value_of(x);
  if (xv <= start) return S(1.0);
  if (xv >= end) return S(0.0);
  return S(0.5) * (S(1.0) - s_sin(S(pi_w) * (x - S(mid))));
}

// height cutoff c_z of the Newtonian cooling at plane k (z_k = z0 + k dz)
__device__ inline double nc_height_cut(const KParams& p, int k) {
  return p.nc_tau == 0.0 ? 0.0
                         : sine_cutoff(zk(p, k), p.nc_z0, p.nc_z1, p.nc_zm, p.nc_pi_zw);
}

// the initial profiles of the Newtonian cooling through the kernel parameters
struct ParamNcTable {
  const KParams& p;
  __device__ __forceinline__ double lnrho0(int i) const { return p.nc_tab[i]; }
  __device__ __forceinline__ double lnT0(int i) const { return p.nc_tab[p.nc_n + i]; }
};

// The radiative-loss table (breakpoints ln T_i, values ln Lambda_i and the
// slopes between them) as read from the kernel parameters; a kernel may pass
// an accessor of its own copy instead (same interface).
struct ParamRadTable {
  const KParams& p;
  __device__ __forceinline__ double lnT(int i) const { return p.rad_lnT[i]; }
  __device__ __forceinline__ double lnL(int i) const { return p.rad_lnL[i]; }
  __device__ __forceinline__ double slope(int i) const { return p.rad_slope[i]; }
};

// continuous piecewise-linear ln Lambda(ln T): segment index (constant
// outside the table, handled by the caller)
template <class Tab>
__device__ __forceinline__ int rad_segment(const Tab& t, int n, double x) {
  int i = 0;
  for (int j = 1; j < n - 1; ++j) i = (x >= t.lnT(j)) ? j : i;
  return i;
}

#define CMHD_FENCE() __builtin_amdgcn_sched_barrier(0)

// what the fluid equations need of the magnetic part
template <typename S>
struct MagState {
  S b[3], iBn;     // field direction and 1/|B|_r (Spitzer)
  S vv[3], sbb;    // b_i d_i B_j and b.vv (Spitzer curvature terms)
  S JxB[3], ohm;   // Lorentz force, eta mu0 J^2 / mu0
};

// Induction equation (out[AX..AZ]) and the magnetic quantities of the fluid
// equations.  Each component of A is read as its gradient and Hessian at
// once (src.gh), and B = curl A + B_ext, div A, d_j B_i and lap A are
// accumulated component by component:
//   B_x = d_y A_z - d_z A_y,  B_y = d_z A_x - d_x A_z,  B_z = d_x A_y - d_y A_x
template <typename S, class Src>
__device__ __forceinline__ void rhs_magnetic(const Src& src, const PointCtx<S>& pc,
                                             const KParams& p, S out[NF], MagState<S>& m) {
  const S w = S(pc.w), dw = S(pc.dw);
  S B[3] = {S(0.0), S(0.0), S(0.0)}, divA = S(0.0);
  S dB[3][3], lapA[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lapA[i] = S(0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j) dB[i][j] = S(0.0);
  }
#pragma unroll(Src::kUnrollA)
  for (int c = 0; c < 3; ++c) {
    S g[3], h[6];
    src.gh(AX + c, g, h);
    // the entries component c reaches (c is uniform across the wave: scalar
    // branches, and no arithmetic on the entries it does not reach)
    const S lap = h[0] + h[1] + h[2];
    if (c == 0) {
      divA = divA + g[0];
      B[1] = B[1] + g[2];
      B[2] = B[2] - g[1];
      lapA[0] = lap;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        dB[1][j] = dB[1][j] + h[hslot(j, 2)];
        dB[2][j] = dB[2][j] - h[hslot(j, 1)];
      }
    } else if (c == 1) {
      divA = divA + g[1];
      B[0] = B[0] - g[2];
      B[2] = B[2] + g[0];
      lapA[1] = lap;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        dB[0][j] = dB[0][j] - h[hslot(j, 2)];
        dB[2][j] = dB[2][j] + h[hslot(j, 0)];
      }
    } else {
      divA = divA + g[2];
      B[0] = B[0] + g[1];
      B[1] = B[1] - g[0];
      lapA[2] = lap;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        dB[0][j] = dB[0][j] + h[hslot(j, 1)];
        dB[1][j] = dB[1][j] - h[hslot(j, 0)];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) B[i] = B[i] + S(p.Bext[i]);
  const S cB[3] = {dB[2][1] - dB[1][2], dB[0][2] - dB[2][0], dB[1][0] - dB[0][1]};  // mu0 J
  {
    const S ux = src.v(UX), uy = src.v(UY), uz = src.v(UZ);
    const S uxB[3] = {uy * B[2] - uz * B[1], uz * B[0] - ux * B[2], ux * B[1] - uy * B[0]};
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out[AX + c] = uxB[c] - S(p.eta) * cB[c] + S(p.eta_s) * w * lapA[c];
    out[AZ] = out[AZ] + S(p.eta_s) * dw * divA;
  }
  // field direction and the curvature terms of the Spitzer flux
  S b[3] = {S(0.0), S(0.0), S(0.0)}, iBn = S(0.0), vv[3] = {S(0.0), S(0.0), S(0.0)};
  S sbb = S(0.0);
  if (p.kappa0 != 0.0) {
    iBn = s_rsqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2] + S(p.B_floor2));
#pragma unroll
    for (int i = 0; i < 3; ++i) b[i] = B[i] * iBn;
#pragma unroll
    for (int j = 0; j < 3; ++j) vv[j] = b[0] * dB[j][0] + b[1] * dB[j][1] + b[2] * dB[j][2];
    sbb = b[0] * vv[0] + b[1] * vv[1] + b[2] * vv[2];
  }
  const S ohm = S(p.eta) * (cB[0] * cB[0] + cB[1] * cB[1] + cB[2] * cB[2]) * S(p.inv_mu0);
  const S J[3] = {cB[0] * S(p.inv_mu0), cB[1] * S(p.inv_mu0), cB[2] * S(p.inv_mu0)};
  const S JxB[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2],
                    J[0] * B[1] - J[1] * B[0]};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    m.b[i] = b[i];
    m.vv[i] = vv[i];
    m.JxB[i] = JxB[i];
  }
  m.iBn = iBn;
  m.sbb = sbb;
  m.ohm = ohm;
}

// The pointwise thermodynamic values the parts of the right-hand side share,
// formed once per zone: T, 1/rho and 1/(c_v T) (float path: from the float64
// state, since ln rho ~ 20 and ln T ~ 14 carry too few bits in float).
template <typename S>
struct PointVals {
  S T, irho, icvT;
};

// T and 1/(c_v T); 1/rho (the two halves of point_vals, which a kernel may
// form on different waves)
template <typename S, class Src>
__device__ __forceinline__ void point_temperature(const Src& src, const KParams& p, S& T,
                                                  S& icvT) {
  if constexpr (std::is_same<S, float>::value) {
    const double T64 = exp(src.v64(LT));
    T = float(T64);
    icvT = float(p.inv_cv / T64);
  } else {
    T = s_exp(src.v(LT));
    icvT = S(p.inv_cv) / T;
  }
}

template <typename S, class Src>
__device__ __forceinline__ S point_irho(const Src& src) {
  if constexpr (std::is_same<S, float>::value) return float(exp(-src.v64(LR)));
  else return s_exp(-src.v(LR));
}

template <typename S, class Src>
__device__ __forceinline__ PointVals<S> point_vals(const Src& src, const KParams& p) {
  PointVals<S> pv;
  point_temperature<S>(src, p, pv.T, pv.icvT);
  pv.irho = point_irho<S>(src);
  return pv;
}

// The terms of the fluid equations that need the magnetic part or the
// Hessian of ln T, in two pieces: rhs_lorentz gives J x B / rho (momentum),
// rhs_heating (eta mu0 J^2 / mu0) / (rho c_v T) + Q_cond / (rho c_v T)
// + chi_s w lap ln T (energy in ln T, Sect. 3 and eq. 19).  Spitzer, with G,
// H the gradient and Hessian of ln T and b = B/|B|_r:
//   Q_cond / (rho c_v T) = (kappa0 T^5/2 / (rho c_v))
//       [7/2 (b.G)^2 + b b:H + (b_i d_i B_j G_j - 2 (b.G) b_i b_k d_i B_k) / |B|_r]
// (the float path forms the coefficient kappa0 T^5/2 / (rho c_v) in float64).
template <typename S>
__device__ __forceinline__ void rhs_lorentz(const MagState<S>& m, const PointVals<S>& pv,
                                            S add[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) add[i] = m.JxB[i] * pv.irho;
}

template <typename S, class Src>
__device__ __forceinline__ S rhs_heating(const Src& src, const PointCtx<S>& pc,
                                         const KParams& p, const MagState<S>& m,
                                         const PointVals<S>& pv) {
  constexpr bool kFloat = std::is_same<S, float>::value;
  S e = m.ohm * pv.irho * pv.icvT;
  const bool swamp_T = p.chi_s != 0.0 && pc.w != 0.0;
  if (p.kappa0 != 0.0 || swamp_T) {
    S G[3], H[6];
    src.gh(LT, G, H);
    if (p.kappa0 != 0.0) {
      const S* b = m.b;
      const S* vv = m.vv;
      const S bG = b[0] * G[0] + b[1] * G[1] + b[2] * G[2];
      const S bbH = b[0] * b[0] * H[0] + b[1] * b[1] * H[1] + b[2] * b[2] * H[2] +
                    S(2.0) * (b[0] * b[1] * H[3] + b[0] * b[2] * H[4] + b[1] * b[2] * H[5]);
      const S vG = vv[0] * G[0] + vv[1] * G[1] + vv[2] * G[2];
      const S bracket = S(3.5) * bG * bG + bbH + (vG - S(2.0) * bG * m.sbb) * m.iBn;
      S kc;
      if constexpr (kFloat) {
        kc = float(p.kappa0 * exp(2.5 * src.v64(LT) - src.v64(LR)) * p.inv_cv);   // FP64 coefficient
      } else {
        // T^{5/2} / rho from the T and 1/rho of the zone (no further exp)
        kc = S(p.kappa0) * (pv.T * pv.T * pv.T * s_rsqrt(pv.T)) * pv.irho * S(p.inv_cv);
      }
      e = e + kc * bracket;
    }
    if (swamp_T) e = e + S(p.chi_s) * S(pc.w) * (H[0] + H[1] + H[2]);
  }
  return e;
}

template <typename S, class Src>
__device__ __forceinline__ void rhs_mag_to_fluid(const Src& src, const PointCtx<S>& pc,
                                                 const KParams& p, const MagState<S>& m,
                                                 const PointVals<S>& pv, S add[4]) {
  rhs_lorentz<S>(m, pv, add);
  add[3] = rhs_heating<S>(src, pc, p, m, pv);
}

// optically thin loss Q_rad/(rho c_v T) = exp(ln rho + lnL(ln T) - ln T) W(ln T) / c_v
// (the only table lookup of the right-hand side)
template <typename S, class Src, class Tab>
__device__ __forceinline__ S rhs_radiation(const Src& src, const KParams& p, const Tab& tab) {
  constexpr bool kFloat = std::is_same<S, float>::value;
  S rad = S(0.0);
  if (p.n_rad > 0) {
    const double x = src.v64(LT);
    if (x > p.lnT_rad_lo) {
      const int n = p.n_rad;
      const int i = rad_segment(tab, n, x);
      const bool below = x < tab.lnT(0), above = x >= tab.lnT(n - 1);
      S wc;
      if (x >= p.lnT_rad_hi) {
        wc = S(1.0);
      } else {
        const S s = (src.v(LT) - S(p.lnT_rad_lo)) * S(p.inv_dlnT_rad);
        wc = s * s * (S(3.0) - S(2.0) * s);
      }
      S ex;
      if constexpr (kFloat) {
        const double lnL64 = below ? tab.lnL(0)
                             : above ? tab.lnL(n - 1)
                                     : tab.lnL(i) + tab.slope(i) * (x - tab.lnT(i));
        ex = float(src.v64(LR) + lnL64 - x);
      } else {
        const S lnL = below   ? S(tab.lnL(0))
                      : above ? S(tab.lnL(n - 1))
                              : S(tab.lnL(i)) + S(tab.slope(i)) * (src.v(LT) - S(tab.lnT(i)));
        ex = src.v(LR) + lnL - src.v(LT);
      }
      rad = s_exp(ex) * wc * S(p.inv_cv);
    }
  }
  return rad;
}

// Chromospheric Newtonian cooling (Sect. 3.1): contribution to d ln T/dt,
// -tau_t c_rho c_z (1 - T*/T) with ln T* = (ln T0(z) + ln T'(rho)) / 2 and
// ln T'(rho) = ln T0(z') where ln rho0(z') = ln rho, linear between the
// bracketing nodes of the (decreasing) ln rho0 table, clamped outside it.  The
// bracket is found on the value (binary search); the interpolation and the
// cutoffs are in S, so that dual numbers carry the derivative.  The float
// path evaluates it in double from the double state.
template <typename S, class Src, class Tab>
__device__ __forceinline__ S rhs_newton(const Src& src, const KParams& p, const Tab& tab,
                                        const PointCtx<S>& pc) {
  if (p.nc_tau == 0.0 || pc.nc_cz == 0.0) return S(0.0);
  constexpr bool kFloat = std::is_same<S, float>::value;
  using T = typename std::conditional<kFloat, double, S>::type;
  T lr, lT;
  if constexpr (kFloat) {
    lr = src.v64(LR);
    lT = src.v64(LT);
  } else {
    lr = src.v(LR);
    lT = src.v(LT);
  }
  const double xv = value_of(lr);
  const T crho = sine_cutoff(T(p.nc_lnrho_phot) - lr, p.nc_dlr0, p.nc_dlr1, p.nc_dlrm,
                               p.nc_pi_dlrw);
  if (value_of(crho) == 0.0) return S(0.0);
  const int n = p.nc_n;
  T lTp;
  if (xv >= tab.lnrho0(0)) {
    lTp = T(tab.lnT0(0));
  } else if (xv <= tab.lnrho0(n - 1)) {
    lTp = T(tab.lnT0(n - 1));
  } else {
    int lo = 0, hi = n - 1;   // lnrho0(lo) >= xv > lnrho0(hi)
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tab.lnrho0(mid) >= xv) lo = mid;
      else hi = mid;
    }
    const double x0 = tab.lnrho0(lo), x1 = tab.lnrho0(lo + 1);
    const double y0 = tab.lnT0(lo), y1 = tab.lnT0(lo + 1);
    const T w = (T(x0) - lr) / T(x0 - x1);
    lTp = T(y0) + w * T(y1 - y0);
  }
  const T lTs = T(0.5) * (T(pc.nc_lnT0) + lTp);
  const T term = T(-p.nc_tau * pc.nc_cz) * crho * (T(1.0) - s_exp(lTs - lT));
  if constexpr (kFloat) return float(term);
  else return term;
}

// Momentum without the Lorentz force:
//   du/dt = -(u.grad)u - R T grad(ln rho + ln T) + g e_z
//           + nu (lap u + grad div u / 3 + 2 S.grad ln rho)
// and the two scalars of the velocity gradient the other equations need,
// div u and S:S (S the traceless rate of strain).  The gradient a_ij = d_j u_i
// is streamed component by component (few values alive): with G = grad ln rho,
//   2 (S.G)_i = sum_j a_ij G_j + sum_j a_ji G_j - 2/3 div u G_i,
//   S:S = 1/2 sum_ij a_ij^2 + 1/2 sum_ij a_ij a_ji - (div u)^2 / 3,
// and grad div u takes the c-th Hessian column of u_c.
template <typename S, class Src>
__device__ __forceinline__ void rhs_momentum(const Src& src, const KParams& p,
                                             const PointVals<S>& pv, S out[NF], S& divu_out,
                                             S& SS_out) {
  const S u[3] = {src.v(UX), src.v(UY), src.v(UZ)};
  S Glr[3], GlT[3];
  src.grad(LR, Glr);
  src.grad(LT, GlT);
  S mom[3], divu = S(0.0), sq = S(0.0), cross = S(0.0);
  S a01 = S(0.0), a02 = S(0.0), a12 = S(0.0);   // a_01, a_02, a_12 for the cross sum
  {
    const S RT = S(p.R) * pv.T;
#pragma unroll
    for (int i = 0; i < 3; ++i) mom[i] = -RT * (Glr[i] + GlT[i]);
  }
#pragma unroll(Src::kUnrollU)
  for (int c = 0; c < 3; ++c) {
    S g[3], h[6];
    src.gh(UX + c, g, h);   // g[j] = a_cj
    // advection, the Laplacian of u_c and sum_j a_cj G_j (into mom[c])
    const S own = -(u[0] * g[0] + u[1] * g[1] + u[2] * g[2]) +
                  S(p.nu) * (h[0] + h[1] + h[2] + g[0] * Glr[0] + g[1] * Glr[1] + g[2] * Glr[2]);
    // the component's own entries (c is uniform across the wave: scalar
    // branches): own into mom[c], div u, G_c = d_c ln rho, the c-th Hessian
    // column hc for grad div u, and a_ij a_ji (the diagonal now, the
    // off-diagonal pairs as their second member arrives)
    S Gc, hc[3];
    sq = sq + (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (c == 0) {
      mom[0] = mom[0] + own;
      divu = divu + g[0];
      Gc = Glr[0];
      hc[0] = h[0];
      hc[1] = h[3];
      hc[2] = h[4];
      cross = cross + g[0] * g[0];
      a01 = g[1];
      a02 = g[2];
    } else if (c == 1) {
      mom[1] = mom[1] + own;
      divu = divu + g[1];
      Gc = Glr[1];
      hc[0] = h[3];
      hc[1] = h[1];
      hc[2] = h[5];
      cross = cross + g[1] * g[1] + S(2.0) * g[0] * a01;
      a12 = g[2];
    } else {
      mom[2] = mom[2] + own;
      divu = divu + g[2];
      Gc = Glr[2];
      hc[0] = h[4];
      hc[1] = h[5];
      hc[2] = h[2];
      cross = cross + g[2] * g[2] + S(2.0) * (g[0] * a02 + g[1] * a12);
    }
    // grad div u (d_i d_c u_c) and a_ci G_c into component i
#pragma unroll
    for (int i = 0; i < 3; ++i)
      mom[i] = mom[i] + S(p.nu) * (hc[i] * S(1.0 / 3.0) + g[i] * Gc);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    out[UX + i] = mom[i] - S(p.nu) * S(2.0 / 3.0) * divu * Glr[i];
  out[UZ] = out[UZ] + S(p.g_z);
  divu_out = divu;
  SS_out = S(0.5) * (sq + cross) - divu * divu * S(1.0 / 3.0);
}

// Continuity in ln rho (Sect. 2.5, eq. 20) and energy in ln T without the
// Ohmic, conductive and swamp terms (those come from rhs_mag_to_fluid):
//   dlnrho = -u.grad ln rho - div u + (D_rho + chi_rho w) lap ln rho + D_rho |grad ln rho|^2
//   dlnT   = -u.grad ln T - (gamma-1) div u + 2 rho nu S:S / (rho c_v T) - Q_rad/(rho c_v T)
//            (+ Newtonian cooling)
// with div u and S:S from rhs_momentum.  In two pieces: rhs_scalars_pre needs
// no velocity gradient (LRp, LTp the two equations without their div u and
// S:S terms), rhs_scalars_post adds those terms.
template <typename S, class Src>
__device__ __forceinline__ void rhs_scalars_pre(const Src& src, const PointCtx<S>& pc,
                                                const KParams& p, S nc, S& LRp, S& LTp) {
  const S u[3] = {src.v(UX), src.v(UY), src.v(UZ)};
  {
    S Glr[3];
    src.grad(LR, Glr);
    const S udr = u[0] * Glr[0] + u[1] * Glr[1] + u[2] * Glr[2];
    const S gr2 = Glr[0] * Glr[0] + Glr[1] * Glr[1] + Glr[2] * Glr[2];
    LRp = (S(p.D_rho) + S(p.chi_rho) * S(pc.w)) * src.lapr() - udr + S(p.D_rho) * gr2;
  }
  {
    S GlT[3];
    src.grad(LT, GlT);
    const S udT = u[0] * GlT[0] + u[1] * GlT[1] + u[2] * GlT[2];
    LTp = nc - udT;
  }
}

// 2 nu S:S / (c_v T) = (2 nu / (c_v T)) S:S
template <typename S>
__device__ __forceinline__ void rhs_scalars_post(const KParams& p, const PointVals<S>& pv, S LRp,
                                                 S LTp, S divu, S SS, S rad, S& dlr, S& dlT) {
  dlr = LRp - divu;
  dlT = S(2.0 * p.nu) * pv.icvT * SS + LTp - rad - S(p.gm1) * divu;
}

template <typename S, class Src>
__device__ __forceinline__ void rhs_scalars(const Src& src, const PointCtx<S>& pc,
                                            const KParams& p, const PointVals<S>& pv, S divu,
                                            S SS, S rad, S nc, S out[NF]) {
  S LRp, LTp;
  rhs_scalars_pre<S>(src, pc, p, nc, LRp, LTp);
  rhs_scalars_post<S>(p, pv, LRp, LTp, divu, SS, rad, out[LR], out[LT]);
}

// the fluid equations without the magnetic terms: momentum, continuity, energy
template <typename S, class Src>
__device__ __forceinline__ void rhs_fluid_core(const Src& src, const PointCtx<S>& pc,
                                               const KParams& p, const PointVals<S>& pv, S rad,
                                               S nc, S out[NF]) {
  S divu, SS;
  rhs_momentum<S>(src, p, pv, out, divu, SS);
  rhs_scalars<S>(src, pc, p, pv, divu, SS, rad, nc, out);
}

// the magnetic part's contributions added to the fluid equations
template <typename S>
__device__ __forceinline__ void rhs_add_magnetic(const S add[4], S out[NF]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) out[UX + i] = out[UX + i] + add[i];
  out[LT] = out[LT] + add[3];
}

// photospheric nudging of A_h toward A_h* (magnetic equations)
template <typename S, class Src>
__device__ __forceinline__ void rhs_boundary_magnetic(const Src& src, const PointCtx<S>& pc,
                                                      const KParams& p, S out[NF]) {
  if (pc.bottom) {
    out[AX] = out[AX] - S(p.tau_A) * (src.v(AX) - pc.ah[0]);
    out[AY] = out[AY] - S(p.tau_A) * (src.v(AY) - pc.ah[1]);
  }
}

// photospheric nudging of u_h toward s(t) u* (eq. 5) and the boundary
// points: u_z = 0 at both boundary planes, ln rho fixed at the photosphere
template <typename S, class Src>
__device__ __forceinline__ void rhs_boundary_fluid(const Src& src, const PointCtx<S>& pc,
                                                   const KParams& p, S out[NF]) {
  if (pc.bottom) {
    out[UX] = out[UX] - S(p.tau_u) * (src.v(UX) - S(pc.ramp) * pc.uh[0]);
    out[UY] = out[UY] - S(p.tau_u) * (src.v(UY) - S(pc.ramp) * pc.uh[1]);
    out[UZ] = S(0.0);
    out[LR] = S(0.0);
  }
  if (pc.top) out[UZ] = S(0.0);
}

// the whole right-hand side at one zone
template <typename S, class Src>
__device__ __forceinline__ void rhs_eval(const Src& src, const PointCtx<S>& pc,
                                         const KParams& p, S out[NF]) {
  MagState<S> m;
  S add[4];
  const S rad = rhs_radiation<S>(src, p, ParamRadTable{p});
  const S nc = rhs_newton<S>(src, p, ParamNcTable{p}, pc);
  const PointVals<S> pv = point_vals<S>(src, p);
  rhs_magnetic<S>(src, pc, p, out, m);
  rhs_mag_to_fluid<S>(src, pc, p, m, pv, add);
  CMHD_FENCE();
  rhs_fluid_core<S>(src, pc, p, pv, rad, nc, out);
  rhs_add_magnetic<S>(add, out);
  rhs_boundary_magnetic<S>(src, pc, p, out);
  rhs_boundary_fluid<S>(src, pc, p, out);
}

}  // namespace cmhd
