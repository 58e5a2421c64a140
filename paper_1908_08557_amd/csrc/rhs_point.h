// Pointwise right-hand side of the MHD system at one zone, from the zone's
// values and its first and second derivatives.  Templated on the scalar type
// S: double (FP64 path), float (split path: derivatives arrive in float,
// the conduction coefficient and the radiative-loss exponent are formed in
// double from the double state) and the forward-mode dual numbers of the
// tangent and adjoint kernels.
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
// div B = 0, and Q_rad = rho^2 Lambda(T) W(T).
#pragma once

#include <type_traits>

#include "cmhd_internal.h"

namespace cmhd {

// Hessian slot of d_i d_j: xx, yy, zz, xy, xz, yz
__host__ __device__ constexpr int hslot(int i, int j) {
  return i == j ? i : (i + j == 1 ? 3 : (i + j == 2 ? 4 : 5));
}

// Inputs of the pointwise right-hand side at one zone.  The second
// derivatives arrive already folded into the combinations the equations use,
// so that fewer values are live at once.
template <typename S>
struct PointIn {
  S v[NF];          // Ax Ay Az ux uy uz lnrho lnT
  S GA[3][3];       // GA[c][d] = d_d A_c
  S dB[3][3];       // dB[i][j] = d_j B_i, from the second derivatives of A
  S lapA[3];        // Laplacian of A_c
  S Gu[3][3];       // Gu[c][d] = d_d u_c
  S lapu[3];        // Laplacian of u_c
  S graddiv[3];     // d_i (div u)
  S Glr[3], GlT[3]; // gradients of ln rho and ln T
  S HT[6];          // Hessian of ln T: xx yy zz xy xz yz
  S lapr;           // Laplacian of ln rho
  double lr64, lT64;  // the FP64 state values of ln rho and ln T (split path)
};

// Fold the six second derivatives h (xx yy zz xy xz yz) of A_c into the
// gradient of B = curl A (dB[i][j] = d_j B_i) and the Laplacian of A_c.
template <typename S>
__host__ __device__ inline void fold_A_hessian(int c, const S h[6], S dB[3][3], S lapA[3]) {
  auto H = [&](int i, int j) -> const S& { return h[hslot(i, j)]; };
  lapA[c] = H(0, 0) + H(1, 1) + H(2, 2);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (c == AX) {          // B_y = d_z A_x - ..., B_z = ... - d_y A_x
      dB[1][j] = dB[1][j] + H(j, 2);
      dB[2][j] = dB[2][j] - H(j, 1);
    } else if (c == AY) {   // B_z = d_x A_y - ..., B_x = ... - d_z A_y
      dB[2][j] = dB[2][j] + H(j, 0);
      dB[0][j] = dB[0][j] - H(j, 2);
    } else {                // B_x = d_y A_z - ..., B_y = ... - d_x A_z
      dB[0][j] = dB[0][j] + H(j, 1);
      dB[1][j] = dB[1][j] - H(j, 0);
    }
  }
}

// Fold the second derivatives of u_c: h holds xx yy zz and the mixed slots
// used by grad div u (xy xz for u_x, xy yz for u_y, xz yz for u_z).
template <typename S>
__host__ __device__ inline void fold_u_hessian(int c, const S h[6], S lapu[3], S graddiv[3]) {
  auto H = [&](int i, int j) -> const S& { return h[hslot(i, j)]; };
  lapu[c] = H(0, 0) + H(1, 1) + H(2, 2);
  // graddiv_i = sum_c d_i d_c u_c
#pragma unroll
  for (int i = 0; i < 3; ++i) graddiv[i] = graddiv[i] + H(i, c);
}

template <typename S>
struct PointCtx {
  double w, dw;       // swamp weight and its z-derivative at this plane
  int bottom, top;    // photospheric / top boundary plane (solar mode)
  S uh[2];            // driver u* at (x, y)
  S ah[2];            // A_h* at (x, y)
  double ramp;        // s(t)
};

// math helpers overloaded on the scalar type
__device__ inline double s_exp(double a) { return exp(a); }
__device__ inline float s_exp(float a) { return expf(a); }
__device__ inline double s_sqrt(double a) { return sqrt(a); }
__device__ inline float s_sqrt(float a) { return __fsqrt_rn(a); }

__device__ inline double value_of(double a) { return a; }
__device__ inline double value_of(float a) { return a; }

// continuous piecewise-linear ln Lambda(ln T): constant outside the table
__device__ inline int rad_segment(const KParams& p, double x) {
  int i = 0;
  for (int j = 1; j < p.n_rad - 1; ++j) i = (x >= p.rad_lnT[j]) ? j : i;
  return i;
}

template <typename S>
__device__ __attribute__((noinline)) void rhs_point(const PointIn<S>& in, const PointCtx<S>& pc, const KParams& p,
                                 S out[NF]) {
  const S* v = in.v;
  auto G = [&](int f, int d) -> S {
    return f < UX ? in.GA[f][d] : (f < LR ? in.Gu[f - UX][d] : (f == LR ? in.Glr[d] : in.GlT[d]));
  };
  auto HT = [&](int i, int j) -> const S& { return in.HT[hslot(i, j)]; };
  auto dB = in.dB;

  // magnetic field B = curl A + B_ext; mu0 J = curl B
  const S B[3] = {G(AZ, 1) - G(AY, 2) + S(p.Bext[0]), G(AX, 2) - G(AZ, 0) + S(p.Bext[1]),
                  G(AY, 0) - G(AX, 1) + S(p.Bext[2])};
  const S cB[3] = {dB[2][1] - dB[1][2], dB[0][2] - dB[2][0], dB[1][0] - dB[0][1]};

  const S ux = v[UX], uy = v[UY], uz = v[UZ];
  S rho, T;
  if constexpr (std::is_same<S, float>::value) {
    rho = float(exp(in.lr64));   // ln rho ~ 20 and ln T ~ 14 carry too few bits in float
    T = float(exp(in.lT64));
  } else {
    rho = s_exp(v[LR]);
    T = s_exp(v[LT]);
  }
  const S irho = S(1.0) / rho;
  const S w = S(pc.w), dw = S(pc.dw);

  // ---- induction, Weyl gauge, with the swamp term of eq. (18)
  const S uxB[3] = {uy * B[2] - uz * B[1], uz * B[0] - ux * B[2], ux * B[1] - uy * B[0]};
  const S divA = G(AX, 0) + G(AY, 1) + G(AZ, 2);
#pragma unroll
  for (int c = 0; c < 3; ++c) out[AX + c] = uxB[c] - S(p.eta) * cB[c] + S(p.eta_s) * w * in.lapA[c];
  out[AZ] = out[AZ] + S(p.eta_s) * dw * divA;

  // ---- momentum
  const S divu = G(UX, 0) + G(UY, 1) + G(UZ, 2);
  S Sij[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Sij[i][j] = S(0.5) * (G(UX + i, j) + G(UX + j, i));
  const S third_div = divu * S(1.0 / 3.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) Sij[i][i] = Sij[i][i] - third_div;
  const S J[3] = {cB[0] * S(p.inv_mu0), cB[1] * S(p.inv_mu0), cB[2] * S(p.inv_mu0)};
  const S JxB[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2],
                    J[0] * B[1] - J[1] * B[0]};
  const S RT = S(p.R) * T;
  const S u[3] = {ux, uy, uz};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const S adv = u[0] * G(UX + i, 0) + u[1] * G(UX + i, 1) + u[2] * G(UX + i, 2);
    const S press = -RT * (G(LR, i) + G(LT, i));
    const S strain = Sij[i][0] * G(LR, 0) + Sij[i][1] * G(LR, 1) + Sij[i][2] * G(LR, 2);
    const S visc = S(p.nu) * (in.lapu[i] + in.graddiv[i] * S(1.0 / 3.0) + S(2.0) * strain);
    out[UX + i] = press - adv + JxB[i] * irho + visc;
  }
  out[UZ] = out[UZ] + S(p.g_z);

  // ---- continuity in ln rho (mass diffusion, Sect. 2.5; swamp eq. 20)
  const S udr = ux * G(LR, 0) + uy * G(LR, 1) + uz * G(LR, 2);
  const S gr2 = G(LR, 0) * G(LR, 0) + G(LR, 1) * G(LR, 1) + G(LR, 2) * G(LR, 2);
  out[LR] = (S(p.D_rho) + S(p.chi_rho) * w) * in.lapr - udr - divu + S(p.D_rho) * gr2;

  // ---- energy in ln T
  const S ohm = S(p.eta) * (cB[0] * cB[0] + cB[1] * cB[1] + cB[2] * cB[2]) * S(p.inv_mu0);
  S SS = S(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) SS = SS + Sij[i][j] * Sij[i][j];
  const S vheat = S(2.0) * rho * S(p.nu) * SS;
  const S heat = (ohm + vheat) * irho / (S(p.cv) * T);

  // Spitzer: Q_cond/(rho c_v T) = [kappa0 T^5/2/(rho c_v)] *
  //   [7/2 (b.G)^2 + b b:H + (b_i d_i B_j G_j - 2 (b.G) b_i b_k d_i B_k) / |B|_r]
  S cond = S(0.0);
  if (p.kappa0 != 0.0) {
    const S Bn = s_sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2] + S(p.B_floor2));
    const S iBn = S(1.0) / Bn;
    const S b[3] = {B[0] * iBn, B[1] * iBn, B[2] * iBn};
    const S bG = b[0] * G(LT, 0) + b[1] * G(LT, 1) + b[2] * G(LT, 2);
    S bbH = S(0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) bbH = bbH + b[i] * b[j] * HT(i, j);
    S vv[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) vv[j] = b[0] * dB[j][0] + b[1] * dB[j][1] + b[2] * dB[j][2];
    const S vG = vv[0] * G(LT, 0) + vv[1] * G(LT, 1) + vv[2] * G(LT, 2);
    const S sbb = b[0] * vv[0] + b[1] * vv[1] + b[2] * vv[2];
    const S bracket = S(3.5) * bG * bG + bbH + (vG - S(2.0) * bG * sbb) * iBn;
    S kc;
    if constexpr (std::is_same<S, float>::value) {
      kc = float(p.kappa0 * exp(2.5 * in.lT64 - in.lr64) / p.cv);   // FP64 coefficient
    } else {
      kc = S(p.kappa0) * s_exp(S(2.5) * v[LT] - v[LR]) * S(1.0 / p.cv);
    }
    cond = kc * bracket;
  }

  // optically thin loss: Q_rad/(rho c_v T) = exp(ln rho + lnL(ln T) - ln T) W(ln T) / c_v
  S rad = S(0.0);
  if (p.n_rad > 0) {
    double x;
    if constexpr (std::is_same<S, float>::value || std::is_same<S, double>::value) {
      x = in.lT64;
    } else {
      x = value_of(v[LT]);
    }
    if (x > p.lnT_rad_lo) {
      int i = rad_segment(p, x);
      S lnL;
      if (x < p.rad_lnT[0]) {
        lnL = S(p.rad_lnL[0]);
      } else if (x >= p.rad_lnT[p.n_rad - 1]) {
        lnL = S(p.rad_lnL[p.n_rad - 1]);
      } else {
        lnL = S(p.rad_lnL[i]) + S(p.rad_slope[i]) * (v[LT] - S(p.rad_lnT[i]));
      }
      S wc;
      if (x >= p.lnT_rad_hi) {
        wc = S(1.0);
      } else {
        const S s = (v[LT] - S(p.lnT_rad_lo)) * S(p.inv_dlnT_rad);
        wc = s * s * (S(3.0) - S(2.0) * s);
      }
      S ex;
      if constexpr (std::is_same<S, float>::value) {
        double lnL64 = (x < p.rad_lnT[0]) ? p.rad_lnL[0]
                       : (x >= p.rad_lnT[p.n_rad - 1])
                           ? p.rad_lnL[p.n_rad - 1]
                           : p.rad_lnL[i] + p.rad_slope[i] * (x - p.rad_lnT[i]);
        ex = float(in.lr64 + lnL64 - x);
      } else {
        ex = v[LR] + lnL - v[LT];
      }
      rad = s_exp(ex) * wc * S(1.0 / p.cv);
    }
  }

  const S udT = ux * G(LT, 0) + uy * G(LT, 1) + uz * G(LT, 2);
  const S lapT = HT(0, 0) + HT(1, 1) + HT(2, 2);
  out[LT] = heat + cond - rad - udT - S(p.gm1) * divu + S(p.chi_s) * w * lapT;

  // ---- photospheric nudging (eq. 5 and the magnetic nudging) and the
  //      closed/'fg' boundary points
  if (pc.bottom) {
    out[UX] = out[UX] - S(p.tau_u) * (ux - S(pc.ramp) * pc.uh[0]);
    out[UY] = out[UY] - S(p.tau_u) * (uy - S(pc.ramp) * pc.uh[1]);
    out[AX] = out[AX] - S(p.tau_A) * (v[AX] - pc.ah[0]);
    out[AY] = out[AY] - S(p.tau_A) * (v[AY] - pc.ah[1]);
    out[UZ] = S(0.0);
    out[LR] = S(0.0);
  }
  if (pc.top) out[UZ] = S(0.0);
}

}  // namespace cmhd
