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
//   S v(f); double v64(f); S d(f, dir); S h(f, slot); S lapr();
//   kUnrollA, kUnrollU: unroll factors of the component loops over A and u
//   (1 keeps a source's on-demand reads in a rolled loop).
// h(f, slot) is only asked for the slots the equations use.
//
// The evaluation is split into a magnetic part (the only one that reads A's
// derivatives) and a fluid part, so that a kernel can release its staged
// copy of A between the two; rhs_eval runs both.
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
__device__ inline double s_sin(double a) { return sin(a); }
__device__ inline double value_of(double a) { return a; }

// 1 for x <= start, 0 for x >= start + width, 1/2 [1 - sin(pi (x - start -
// width/2) / width)] between (the sine cutoffs of the Newtonian cooling)
template <typename S>
__device__ inline S sine_cutoff(S x, double start, double width) {
  const double xv = value_of(x);
  if (xv <= start) return S(1.0);
  if (xv >= start + width) return S(0.0);
  return S(0.5) * (S(1.0) - s_sin(S(M_PI / width) * (x - S(start + 0.5 * width))));
}

// height cutoff c_z of the Newtonian cooling at plane k (z_k = z0 + k dz)
__device__ inline double nc_height_cut(const KParams& p, int k) {
  return p.nc_tau == 0.0 ? 0.0 : sine_cutoff(zk(p, k), p.nc_z0, p.nc_zw);
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

// what the fluid part needs of the magnetic part
template <typename S>
struct MagState {
  S b[3], iBn;     // field direction and 1/|B|_r (Spitzer)
  S vv[3], sbb;    // b_i d_i B_j and b.vv (Spitzer curvature terms)
  S JxB[3], ohm;   // Lorentz force, eta mu0 J^2 / mu0
};

template <typename S, class Src>
__device__ __forceinline__ void rhs_magnetic(const Src& src, const PointCtx<S>& pc,
                                             const KParams& p, S out[NF], MagState<S>& m) {
  const S w = S(pc.w), dw = S(pc.dw);
  const S ux = src.v(UX), uy = src.v(UY), uz = src.v(UZ);

  // ================= magnetic phase: B, grad B, induction ===================
  S B[3], divA;
  {
    const S Axy = src.d(AX, 1), Axz = src.d(AX, 2), Ayx = src.d(AY, 0);
    const S Ayz = src.d(AY, 2), Azx = src.d(AZ, 0), Azy = src.d(AZ, 1);
    B[0] = Azy - Ayz + S(p.Bext[0]);
    B[1] = Axz - Azx + S(p.Bext[1]);
    B[2] = Ayx - Axy + S(p.Bext[2]);
    divA = src.d(AX, 0) + src.d(AY, 1) + src.d(AZ, 2);
  }
  // dB[i][j] = d_j B_i from the second derivatives of A (each mixed one read once):
  //   B_x = d_y A_z - d_z A_y,  B_y = d_z A_x - d_x A_z,  B_z = d_x A_y - d_y A_x
  S dB[3][3], lapA[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dB[i][j] = S(0.0);
  // a rolled loop over the components when the source allows it: each
  // component's stencil reads then form their own scheduling region
#pragma unroll(Src::kUnrollA)
  for (int c = 0; c < 3; ++c) {
    S h[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) h[s] = src.h(AX + c, s);
    const S lap = h[0] + h[1] + h[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) lapA[i] = (i == c) ? lap : lapA[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const S hj0 = h[hslot(j, 0)], hj1 = h[hslot(j, 1)], hj2 = h[hslot(j, 2)];
      dB[0][j] = dB[0][j] + (c == AY ? -hj2 : (c == AZ ? hj1 : S(0.0)));
      dB[1][j] = dB[1][j] + (c == AX ? hj2 : (c == AZ ? -hj0 : S(0.0)));
      dB[2][j] = dB[2][j] + (c == AX ? -hj1 : (c == AY ? hj0 : S(0.0)));
    }
  }
  const S cB[3] = {dB[2][1] - dB[1][2], dB[0][2] - dB[2][0], dB[1][0] - dB[0][1]};  // mu0 J
  {
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
    const S Bn = s_sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2] + S(p.B_floor2));
    iBn = S(1.0) / Bn;
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
      rad = s_exp(ex) * wc * S(1.0 / p.cv);
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
  const T crho = sine_cutoff(T(p.nc_lnrho_phot) - lr, p.nc_dlr0, p.nc_dlrw);
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

template <typename S, class Src>
__device__ __forceinline__ void rhs_fluid(const Src& src, const PointCtx<S>& pc,
                                          const KParams& p, const MagState<S>& m, S rad,
                                          S nc, S out[NF]) {
  constexpr bool kFloat = std::is_same<S, float>::value;
  const S w = S(pc.w);
  const S ux = src.v(UX), uy = src.v(UY), uz = src.v(UZ);
  const S* JxB = m.JxB;
  const S* b = m.b;
  const S* vv = m.vv;
  const S iBn = m.iBn, sbb = m.sbb, ohm = m.ohm;

  // ================= momentum ===============================================
  S rho, T;
  if constexpr (kFloat) {
    rho = float(exp(src.v64(LR)));   // ln rho ~ 20 and ln T ~ 14 carry too few bits in float
    T = float(exp(src.v64(LT)));
  } else {
    rho = s_exp(src.v(LR));
    T = s_exp(src.v(LT));
  }
  const S irho = S(1.0) / rho;
  const S Glr[3] = {src.d(LR, 0), src.d(LR, 1), src.d(LR, 2)};
  const S GlT[3] = {src.d(LT, 0), src.d(LT, 1), src.d(LT, 2)};
  S divu, SS;
  {
    S Gu[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) Gu[c][d] = src.d(UX + c, d);
    divu = Gu[0][0] + Gu[1][1] + Gu[2][2];
    S Sij[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Sij[i][j] = S(0.5) * (Gu[i][j] + Gu[j][i]);
    const S third_div = divu * S(1.0 / 3.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) Sij[i][i] = Sij[i][i] - third_div;
    SS = S(0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) SS = SS + Sij[i][j] * Sij[i][j];
    // Laplacian of u_c and grad div u (mixed slots: xy, xz for u_x; xy, yz
    // for u_y; xz, yz for u_z)
    S lapu[3], gd[3] = {S(0.0), S(0.0), S(0.0)};
#pragma unroll(Src::kUnrollU)
    for (int c = 0; c < 3; ++c) {
      const S hxx = src.h(UX + c, 0), hyy = src.h(UX + c, 1), hzz = src.h(UX + c, 2);
      const S lap = hxx + hyy + hzz;
      // mixed slots of grad div u: xy for u_x, u_y; xz for u_x, u_z; yz for u_y, u_z
      const S m1 = src.h(UX + c, c == 0 ? 3 : (c == 1 ? 3 : 4));   // xy, xy, xz
      const S m2 = src.h(UX + c, c == 0 ? 4 : 5);                  // xz, yz, yz
#pragma unroll
      for (int i = 0; i < 3; ++i) lapu[i] = (i == c) ? lap : lapu[i];
      // gd_i += d_i d_c u_c
      gd[0] = gd[0] + (c == 0 ? hxx : m1);
      gd[1] = gd[1] + (c == 0 ? m1 : (c == 1 ? hyy : m2));
      gd[2] = gd[2] + (c == 2 ? hzz : m2);
    }
    const S RT = S(p.R) * T;
    const S u[3] = {ux, uy, uz};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const S adv = u[0] * Gu[i][0] + u[1] * Gu[i][1] + u[2] * Gu[i][2];
      const S press = -RT * (Glr[i] + GlT[i]);
      const S strain = Sij[i][0] * Glr[0] + Sij[i][1] * Glr[1] + Sij[i][2] * Glr[2];
      const S visc = S(p.nu) * (lapu[i] + gd[i] * S(1.0 / 3.0) + S(2.0) * strain);
      out[UX + i] = press - adv + JxB[i] * irho + visc;
    }
    out[UZ] = out[UZ] + S(p.g_z);
  }
  CMHD_FENCE();

  // ================= continuity in ln rho (Sect. 2.5, eq. 20) ================
  {
    const S udr = ux * Glr[0] + uy * Glr[1] + uz * Glr[2];
    const S gr2 = Glr[0] * Glr[0] + Glr[1] * Glr[1] + Glr[2] * Glr[2];
    out[LR] = (S(p.D_rho) + S(p.chi_rho) * w) * src.lapr() - udr - divu + S(p.D_rho) * gr2;
  }

  // ================= energy in ln T ===========================================
  const S vheat = S(2.0) * rho * S(p.nu) * SS;
  const S heat = (ohm + vheat) * irho / (S(p.cv) * T);
  S lapT, cond = S(0.0);
  {
    const S hxx = src.h(LT, 0), hyy = src.h(LT, 1), hzz = src.h(LT, 2);
    lapT = hxx + hyy + hzz;
    if (p.kappa0 != 0.0) {
      const S hxy = src.h(LT, 3), hxz = src.h(LT, 4), hyz = src.h(LT, 5);
      const S bG = b[0] * GlT[0] + b[1] * GlT[1] + b[2] * GlT[2];
      const S bbH = b[0] * b[0] * hxx + b[1] * b[1] * hyy + b[2] * b[2] * hzz +
                    S(2.0) * (b[0] * b[1] * hxy + b[0] * b[2] * hxz + b[1] * b[2] * hyz);
      const S vG = vv[0] * GlT[0] + vv[1] * GlT[1] + vv[2] * GlT[2];
      const S bracket = S(3.5) * bG * bG + bbH + (vG - S(2.0) * bG * sbb) * iBn;
      S kc;
      if constexpr (kFloat) {
        kc = float(p.kappa0 * exp(2.5 * src.v64(LT) - src.v64(LR)) / p.cv);   // FP64 coefficient
      } else {
        kc = S(p.kappa0) * s_exp(S(2.5) * src.v(LT) - src.v(LR)) * S(1.0 / p.cv);
      }
      cond = kc * bracket;
    }
  }

  {
    const S udT = ux * GlT[0] + uy * GlT[1] + uz * GlT[2];
    out[LT] = heat + cond - rad - udT - S(p.gm1) * divu + S(p.chi_s) * w * lapT + nc;
  }

  // ================= photospheric nudging and boundary points ================
  if (pc.bottom) {
    out[UX] = out[UX] - S(p.tau_u) * (ux - S(pc.ramp) * pc.uh[0]);
    out[UY] = out[UY] - S(p.tau_u) * (uy - S(pc.ramp) * pc.uh[1]);
    out[AX] = out[AX] - S(p.tau_A) * (src.v(AX) - pc.ah[0]);
    out[AY] = out[AY] - S(p.tau_A) * (src.v(AY) - pc.ah[1]);
    out[UZ] = S(0.0);
    out[LR] = S(0.0);
  }
  if (pc.top) out[UZ] = S(0.0);
}

template <typename S, class Src>
__device__ __forceinline__ void rhs_eval(const Src& src, const PointCtx<S>& pc,
                                         const KParams& p, S out[NF]) {
  MagState<S> m;
  const S rad = rhs_radiation<S>(src, p, ParamRadTable{p});
  const S nc = rhs_newton<S>(src, p, ParamNcTable{p}, pc);
  rhs_magnetic<S>(src, pc, p, out, m);
  CMHD_FENCE();
  rhs_fluid<S>(src, pc, p, m, rad, nc, out);
}

}  // namespace cmhd
