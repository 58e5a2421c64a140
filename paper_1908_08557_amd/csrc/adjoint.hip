// Tangent-linear (JVP) and adjoint (VJP) pieces of one RHS evaluation.
//
// The RHS at an interior zone is R = P(q) with q the 72 pointwise inputs
// (values, first derivatives, the second derivatives the equations use, the
// Laplacian of ln rho), q = L(G(X)) linear stencils of the ghost-filled state
// G(X).  Hence
//   JVP:  dR = P'(q) L G'(X) dX                    (one dual-number pass)
//   VJP:  Xbar = G'(X)^T L^T P'(q)^T Rbar          (72 seeded dual passes,
//         transposed stencils, transposed ghost rules)
// The pointwise P is the same templated program as the forward kernel
// (rhs_eval), evaluated on dual numbers; the stencil and ghost transposes are
// written out here.  Correctness, not speed, is the target of these kernels.
#include "launch.h"
#include "dual.h"
#include "qslots.h"
#include "rhs_point.h"

namespace cmhd {

namespace {

constexpr double W1[3] = {45.0, -9.0, 1.0};

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// value of field f of a ghost-filled state at (x, y, array plane kz), x/y wrapped
__device__ __forceinline__ double gval(const KParams& p, const double* g, int f, int x, int y,
                                       int kz) {
  return g[f * p.sfield + (long long)kz * p.splane + (long long)wrapi(y, p.ny) * p.nx +
           wrapi(x, p.nx)];
}

__device__ __forceinline__ double inv60(const KParams& p, int d) {
  return d == 0 ? p.i60dx : (d == 1 ? p.i60dy : p.i60dz);
}
__device__ __forceinline__ double inv180(const KParams& p, int d) {
  return d == 0 ? p.i180dx2 : (d == 1 ? p.i180dy2 : p.i180dz2);
}
__device__ __forceinline__ void step3(int d, int m, int& dx, int& dy, int& dz) {
  dx = d == 0 ? m : 0;
  dy = d == 1 ? m : 0;
  dz = d == 2 ? m : 0;
}

// D1 and D2 along d, and D1_i D1_j, of field f at (x, y, kz)
__device__ double st_d1(const KParams& p, const double* g, int f, int x, int y, int kz, int d) {
  double acc = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int a, b, c;
    step3(d, m, a, b, c);
    acc += W1[m - 1] * (gval(p, g, f, x + a, y + b, kz + c) - gval(p, g, f, x - a, y - b, kz - c));
  }
  // non-uniform z: the plane-index stencil scaled by the metric of plane kz
  if (d == 2 && p.stretched) return acc * p.ztab[zt_c1(p) + kz - NG];
  return acc * inv60(p, d);
}
__device__ double st_d2(const KParams& p, const double* g, int f, int x, int y, int kz, int d) {
  const double W2[3] = {270.0, -27.0, 2.0};
  double acc = -490.0 * gval(p, g, f, x, y, kz);
  double acc1 = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int a, b, c;
    step3(d, m, a, b, c);
    const double hi = gval(p, g, f, x + a, y + b, kz + c), lo = gval(p, g, f, x - a, y - b, kz - c);
    acc += W2[m - 1] * (hi + lo);
    acc1 += W1[m - 1] * (hi - lo);
  }
  // non-uniform z: c2 S2 + c3 S1 at plane kz
  if (d == 2 && p.stretched)
    return acc * p.ztab[zt_c2(p) + kz - NG] + acc1 * p.ztab[zt_c3(p) + kz - NG];
  return acc * inv180(p, d);
}
__device__ double st_mixed(const KParams& p, const double* g, int f, int x, int y, int kz, int i,
                           int j) {
  double acc = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int a, b, c;
    step3(i, m, a, b, c);
    acc += W1[m - 1] * (st_d1(p, g, f, x + a, y + b, kz + c, j) -
                        st_d1(p, g, f, x - a, y - b, kz - c, j));
  }
  return acc * inv60(p, i);
}

__device__ __forceinline__ void hslot_dirs(int s, int& i, int& j) {
  const int I[6] = {0, 1, 2, 0, 0, 1}, J[6] = {0, 1, 2, 1, 2, 2};
  i = I[s];
  j = J[s];
}

// ---------------------------------------------------------------------------
// q = L(G): the 72 pointwise inputs of every interior zone
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_point_q(const KParams p, const double* __restrict__ g, double* __restrict__ Q) {
  const long long nzone = (long long)p.nz * p.splane;
  for (long long z = blockIdx.x * (long long)blockDim.x + threadIdx.x; z < nzone;
       z += (long long)gridDim.x * blockDim.x) {
    const int k = int(z / p.splane);
    const long long col = z - (long long)k * p.splane;
    const int y = int(col / p.nx), x = int(col - (long long)y * p.nx);
    const int kz = k + NG;
    for (int f = 0; f < NF; ++f) {
      Q[q_v(f) * nzone + z] = gval(p, g, f, x, y, kz);
      for (int d = 0; d < 3; ++d) Q[q_d(f, d) * nzone + z] = st_d1(p, g, f, x, y, kz, d);
      for (int s = 0; s < 6; ++s) {
        const int slot = q_h(f, s);
        if (slot < 0) continue;
        int i, j;
        hslot_dirs(s, i, j);
        Q[slot * nzone + z] =
            i == j ? st_d2(p, g, f, x, y, kz, i) : st_mixed(p, g, f, x, y, kz, i, j);
      }
    }
    Q[Q_LAPR * nzone + z] = st_d2(p, g, LR, x, y, kz, 0) + st_d2(p, g, LR, x, y, kz, 1) +
                            st_d2(p, g, LR, x, y, kz, 2);
  }
}

// pointwise inputs from the Q buffer as dual numbers: tangent from dQ (JVP)
// or a unit seed in one slot (one column of the pointwise Jacobian)
struct QSource {
  static constexpr int kUnrollA = 3, kUnrollU = 3;
  const double* Q;
  const double* dQ;   // may be null
  long long nzone, z;
  int seed;           // slot whose tangent is 1 (-1: none)
  __device__ Dual q(int slot) const {
    const double v = Q[slot * nzone + z];
    double d = dQ ? dQ[slot * nzone + z] : 0.0;
    if (slot == seed) d = 1.0;
    return Dual(v, d);
  }
  __device__ Dual v(int f) const { return q(q_v(f)); }
  __device__ double v64(int f) const { return Q[q_v(f) * nzone + z]; }
  __device__ Dual d(int f, int dir) const { return q(q_d(f, dir)); }
  __device__ Dual h(int f, int s) const {
    const int slot = q_h(f, s);
    return slot >= 0 ? q(slot) : Dual(0.0);
  }
  __device__ Dual lapr() const { return q(Q_LAPR); }
  __device__ void grad(int f, Dual g[3]) const {
    for (int i = 0; i < 3; ++i) g[i] = d(f, i);
  }
  __device__ void gh(int f, Dual g[3], Dual hh[6]) const {
    for (int i = 0; i < 3; ++i) g[i] = d(f, i);
    for (int s = 0; s < 6; ++s) hh[s] = h(f, s);
  }
};

__device__ void swamp_at(const KParams& p, int k, double& w, double& dw) {
  w = 0.0;
  dw = 0.0;
  if (!p.solar || (p.eta_s == 0.0 && p.chi_s == 0.0 && p.chi_rho == 0.0)) return;
  const double z = zk(p, k);
  const double L = p.z_t - p.z_s;
  double s = (z - p.z_s) / L;
  s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  w = s * s * (3.0 - 2.0 * s);
  dw = (z > p.z_s && z < p.z_t) ? 6.0 * s * (1.0 - s) / L : 0.0;
}

__device__ PointCtx<Dual> point_ctx(const KParams& p, int k, long long col, const double* uh,
                                    const double* ah, const double* duh, double ramp) {
  PointCtx<Dual> pc;
  swamp_at(p, k, pc.w, pc.dw);
  pc.bottom = p.solar && k == 0;
  pc.top = p.solar && k == p.nz - 1;
  pc.ramp = ramp;
  pc.nc_cz = nc_height_cut(p, k);
  pc.nc_lnT0 = p.nc_tau != 0.0 ? p.nc_tab[p.nc_n + k + NG] : 0.0;
  if (pc.bottom) {
    pc.uh[0] = Dual(uh[col], duh ? duh[col] : 0.0);
    pc.uh[1] = Dual(uh[p.splane + col], duh ? duh[p.splane + col] : 0.0);
    pc.ah[0] = Dual(ah[col]);
    pc.ah[1] = Dual(ah[p.splane + col]);
  } else {
    pc.uh[0] = pc.uh[1] = pc.ah[0] = pc.ah[1] = Dual(0.0);
  }
  return pc;
}

// dR = P'(q) dq (+ driver tangent) at every interior zone, state layout
__global__ __launch_bounds__(128) void k_point_jvp(const KParams p, const double* __restrict__ Q,
                            const double* __restrict__ dQ, const double* __restrict__ uh,
                            const double* __restrict__ ah, const double* __restrict__ duh,
                            double ramp, double* __restrict__ dR) {
  const long long nzone = (long long)p.nz * p.splane;
  for (long long z = blockIdx.x * (long long)blockDim.x + threadIdx.x; z < nzone;
       z += (long long)gridDim.x * blockDim.x) {
    const int k = int(z / p.splane);
    const long long col = z - (long long)k * p.splane;
    QSource src{Q, dQ, nzone, z, -1};
    const PointCtx<Dual> pc = point_ctx(p, k, col, uh, ah, duh, ramp);
    Dual out[NF];
    rhs_eval<Dual>(src, pc, p, out);
    for (int f = 0; f < NF; ++f) dR[f * p.sfield + NG * p.splane + z] = out[f].d;
  }
}

// qbar = P'(q)^T Rbar at every interior zone (72 seeded passes); the driver
// cotangent of the photospheric nudging is accumulated into uhbar
__global__ __launch_bounds__(128) void k_point_vjp(const KParams p, const double* __restrict__ Q,
                            const double* __restrict__ Rbar, const double* __restrict__ uh,
                            const double* __restrict__ ah, double ramp,
                            double* __restrict__ Qbar, double* __restrict__ uhbar) {
  const long long nzone = (long long)p.nz * p.splane;
  for (long long z = blockIdx.x * (long long)blockDim.x + threadIdx.x; z < nzone;
       z += (long long)gridDim.x * blockDim.x) {
    const int k = int(z / p.splane);
    const long long col = z - (long long)k * p.splane;
    double rb[NF];
    for (int f = 0; f < NF; ++f) rb[f] = Rbar[f * p.sfield + NG * p.splane + z];
    const PointCtx<Dual> pc = point_ctx(p, k, col, uh, ah, nullptr, ramp);
    for (int i = 0; i < NQ; ++i) {
      QSource src{Q, nullptr, nzone, z, i};
      Dual out[NF];
      rhs_eval<Dual>(src, pc, p, out);
      double acc = 0.0;
      for (int f = 0; f < NF; ++f) acc += rb[f] * out[f].d;
      Qbar[i * nzone + z] = acc;
    }
    if (pc.bottom) {   // d/du* of -tau_u (u_h - s u*)
      uhbar[col] += p.tau_u * ramp * rb[UX];
      uhbar[p.splane + col] += p.tau_u * ramp * rb[UY];
    }
  }
}

// lower ghost rows of u_h: R = -tau_u (u - s u*)
__global__ __launch_bounds__(256) void k_ghost_rows_jvp(const KParams p, const double* __restrict__ dX,
                                 const double* __restrict__ duh, double ramp,
                                 double* __restrict__ dR) {
  const long long n = 2LL * NG * p.splane;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int comp = int(i / (NG * p.splane));
    const long long rem = i - comp * NG * p.splane;
    const long long col = rem % p.splane;
    const long long idx = (UX + comp) * p.sfield + rem;
    dR[idx] = -p.tau_u * (dX[idx] - ramp * (duh ? duh[comp * p.splane + col] : 0.0));
  }
}
__global__ __launch_bounds__(256) void k_ghost_rows_vjp(const KParams p, const double* __restrict__ Rbar, double ramp,
                                 double* __restrict__ Xbar, double* __restrict__ uhbar) {
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < p.splane;
       col += (long long)gridDim.x * blockDim.x) {
    for (int comp = 0; comp < 2; ++comp) {
      double acc = 0.0;
      for (int j = 0; j < NG; ++j) {
        const long long idx = (UX + comp) * p.sfield + (long long)j * p.splane + col;
        Xbar[idx] += -p.tau_u * Rbar[idx];
        acc += Rbar[idx];
      }
      uhbar[comp * p.splane + col] += p.tau_u * ramp * acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Gbar = L^T qbar on the extended grid (interior and z ghosts); qbar is zero
// outside the interior in z and periodic in x, y
// ---------------------------------------------------------------------------
__device__ __forceinline__ double qb(const KParams& p, const double* Qb, int slot, int x, int y,
                                     int k) {
  if (k < 0 || k >= p.nz) return 0.0;
  return Qb[slot * (long long)p.nz * p.splane + (long long)k * p.splane +
            (long long)wrapi(y, p.ny) * p.nx + wrapi(x, p.nx)];
}
// qbar of zone k scaled by the z metric table entry at offset `off` (zero
// outside the interior, as qbar)
__device__ __forceinline__ double qbm(const KParams& p, const double* Qb, int slot, int x, int y,
                                      int k, int off) {
  if (k < 0 || k >= p.nz) return 0.0;
  return p.ztab[off + k] * qb(p, Qb, slot, x, y, k);
}
__device__ double qb_d1(const KParams& p, const double* Qb, int slot, int x, int y, int k, int d) {
  double acc = 0.0;
  if (d == 2 && p.stretched) {
    // (diag(c1) S1)^T = S1^T diag(c1): the metric belongs to the zone of qbar
    const int o1 = zt_c1(p);
    for (int m = 1; m <= 3; ++m)
      acc += W1[m - 1] * (qbm(p, Qb, slot, x, y, k + m, o1) - qbm(p, Qb, slot, x, y, k - m, o1));
    return acc;
  }
  for (int m = 1; m <= 3; ++m) {
    int a, b, c;
    step3(d, m, a, b, c);
    acc += W1[m - 1] * (qb(p, Qb, slot, x + a, y + b, k + c) - qb(p, Qb, slot, x - a, y - b, k - c));
  }
  return acc * inv60(p, d);
}
__device__ double qb_d2(const KParams& p, const double* Qb, int slot, int x, int y, int k, int d) {
  const double W2[3] = {270.0, -27.0, 2.0};
  if (d == 2 && p.stretched) {
    // (diag(c2) S2 + diag(c3) S1)^T = S2 diag(c2) - S1 diag(c3)
    const int o2 = zt_c2(p), o3 = zt_c3(p);
    double acc = -490.0 * qbm(p, Qb, slot, x, y, k, o2);
    for (int m = 1; m <= 3; ++m) {
      acc += W2[m - 1] * (qbm(p, Qb, slot, x, y, k + m, o2) + qbm(p, Qb, slot, x, y, k - m, o2));
      acc -= W1[m - 1] * (qbm(p, Qb, slot, x, y, k + m, o3) - qbm(p, Qb, slot, x, y, k - m, o3));
    }
    return acc;
  }
  double acc = -490.0 * qb(p, Qb, slot, x, y, k);
  for (int m = 1; m <= 3; ++m) {
    int a, b, c;
    step3(d, m, a, b, c);
    acc += W2[m - 1] * (qb(p, Qb, slot, x + a, y + b, k + c) + qb(p, Qb, slot, x - a, y - b, k - c));
  }
  return acc * inv180(p, d);
}
__device__ double qb_mixed(const KParams& p, const double* Qb, int slot, int x, int y, int k, int i,
                           int j) {
  double acc = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int a, b, c;
    step3(i, m, a, b, c);
    acc += W1[m - 1] * (qb_d1(p, Qb, slot, x + a, y + b, k + c, j) -
                        qb_d1(p, Qb, slot, x - a, y - b, k - c, j));
  }
  return acc * inv60(p, i);
}

__global__ __launch_bounds__(128) void k_stencil_T(const KParams p, const double* __restrict__ Qb,
                            double* __restrict__ Gb) {
  const long long n = (long long)(p.nz + 2 * NG) * p.splane;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int kz = int(e / p.splane);
    const long long col = e - (long long)kz * p.splane;
    const int y = int(col / p.nx), x = int(col - (long long)y * p.nx);
    const int k = kz - NG;
    for (int f = 0; f < NF; ++f) {
      double acc = qb(p, Qb, q_v(f), x, y, k);
      for (int d = 0; d < 3; ++d) acc -= qb_d1(p, Qb, q_d(f, d), x, y, k, d);   // D1^T = -D1
      for (int s = 0; s < 6; ++s) {
        const int slot = q_h(f, s);
        if (slot < 0) continue;
        int i, j;
        hslot_dirs(s, i, j);
        // D2^T = D2; (D1_i D1_j)^T has the same product stencil
        acc += i == j ? qb_d2(p, Qb, slot, x, y, k, i) : qb_mixed(p, Qb, slot, x, y, k, i, j);
      }
      if (f == LR)
        acc += qb_d2(p, Qb, Q_LAPR, x, y, k, 0) + qb_d2(p, Qb, Q_LAPR, x, y, k, 1) +
               qb_d2(p, Qb, Q_LAPR, x, y, k, 2);
      Gb[f * p.sfield + e] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// ghost rules: linearisation (JVP) and transpose (VJP)
// ---------------------------------------------------------------------------

// dG = G'(X) dX for the non-Fourier solar rules; X is ghost-filled
__global__ __launch_bounds__(256) void k_fill_solar_columns_lin(const KParams p, const double* __restrict__ g,
                                         double* __restrict__ dg) {
  const long long sp = p.splane;
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < sp;
       col += (long long)gridDim.x * blockDim.x) {
    double* uz = dg + UZ * p.sfield + col;
    double* ux = dg + UX * p.sfield + col;
    double* uy = dg + UY * p.sfield + col;
    double* lr = dg + LR * p.sfield + col;
    double* lT = dg + LT * p.sfield + col;
    const double* lT0 = g + LT * p.sfield + col;
    const int kb = NG, kt = NG + p.nz - 1;
    for (int j = 1; j <= NG; ++j) {
      uz[(kb - j) * sp] = -uz[(kb + j) * sp];
      uz[(kt + j) * sp] = -uz[(kt - j) * sp];
      ux[(kt + j) * sp] = ux[(kt - j) * sp];
      uy[(kt + j) * sp] = uy[(kt - j) * sp];
      lr[(kb - j) * sp] = 0.0;   // density below the photosphere is fixed
    }
    for (int j = 1; j <= NG; ++j) {
      const int up = kb - j + 1;
      const double fac = 1.0 + p.dz_lo[j - 1] * p.g_z / (p.R * exp(lT0[up * sp]));
      lT[(kb - j) * sp] = fac * lT[up * sp] + lr[up * sp] - lr[(kb - j) * sp];
    }
    if (!p.stretched) {
      const double Ttop = exp(lT0[kt * sp]);
      for (int j = 1; j <= NG; ++j) {
        lT[(kt + j) * sp] = lT[(kt - j) * sp];
        lr[(kt + j) * sp] =
            lr[(kt - j) * sp] - p.g_z * (2.0 * j * p.dz) / (p.R * Ttop) * lT[kt * sp];
      }
    } else {
      // eq. (15): lr_j = lr_{j-1} + K_j / (T_{j-1} + T_j), K_j = 2 g dz_hi / R
      for (int j = 1; j <= NG; ++j) lT[(kt + j) * sp] = lT[(kt - j) * sp];
      for (int j = 1; j <= NG; ++j) {
        const double Ta = exp(lT0[(kt + j - 1) * sp]), Tb = exp(lT0[(kt + j) * sp]);
        const double c = -2.0 * p.g_z * p.dz_hi[j - 1] / (p.R * (Ta + Tb) * (Ta + Tb));
        lr[(kt + j) * sp] =
            lr[(kt + j - 1) * sp] + c * (Ta * lT[(kt + j - 1) * sp] + Tb * lT[(kt + j) * sp]);
      }
    }
  }
}

// Xbar += (fold of the solar ghost rules)^T Gbar, except the Fourier part;
// also adds the interior and the u_h ghost rows of Gbar
__global__ __launch_bounds__(256) void k_fold_solar(const KParams p, const double* __restrict__ g,
                             const double* __restrict__ Gb, double* __restrict__ Xb) {
  const long long sp = p.splane;
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < sp;
       col += (long long)gridDim.x * blockDim.x) {
    const int kb = NG, kt = NG + p.nz - 1;
    auto G = [&](int f, int kz) { return Gb[f * p.sfield + kz * sp + col]; };
    auto X = [&](int f, int kz) -> double& { return Xb[f * p.sfield + kz * sp + col]; };
    // interior of every field, and the state rows of u_h below the photosphere
    for (int f = 0; f < NF; ++f)
      for (int kz = kb; kz <= kt; ++kz) X(f, kz) += G(f, kz);
    for (int kz = 0; kz < NG; ++kz) {
      X(UX, kz) += G(UX, kz);
      X(UY, kz) += G(UY, kz);
    }
    // closed boundaries: u_z antisymmetric, u_h symmetric above
    for (int j = 1; j <= NG; ++j) {
      X(UZ, kb + j) -= G(UZ, kb - j);
      X(UZ, kt - j) -= G(UZ, kt + j);
      X(UX, kt - j) += G(UX, kt + j);
      X(UY, kt - j) += G(UY, kt + j);
    }
    // ln T below: reverse the hydrostatic recursion (j = 3, 2, 1)
    double gT[NG + 1];   // running cotangent of ln T at k = 0, -1, -2, -3
    for (int j = 0; j <= NG; ++j) gT[j] = G(LT, kb - j);
    const double* lT0 = g + LT * p.sfield + col;
    for (int j = NG; j >= 1; --j) {
      const int up = kb - j + 1;
      const double fac = 1.0 + p.dz_lo[j - 1] * p.g_z / (p.R * exp(lT0[up * sp]));
      gT[j - 1] += fac * gT[j];
      if (j == 1) X(LR, kb) += gT[j];   // d ln T(-1) / d ln rho(0)
    }
    X(LT, kb) += gT[0] - G(LT, kb);   // the interior value was already added
    if (!p.stretched) {
      // ln T above symmetric; ln rho above hydrostatic mirror (depends on T(nz-1))
      const double Ttop = exp(lT0[kt * sp]);
      for (int j = 1; j <= NG; ++j) {
        X(LT, kt - j) += G(LT, kt + j);
        X(LR, kt - j) += G(LR, kt + j);
        X(LT, kt) += -p.g_z * (2.0 * j * p.dz) / (p.R * Ttop) * G(LR, kt + j);
      }
    } else {
      // reverse the eq. (15) recursion (j = 3, 2, 1): the density cotangent
      // runs down to ln rho(nz-1) and feeds the ln T of both planes of each
      // step; the ghost ln T then folds back by the mirror of eq. (11)
      double gR = 0.0;
      double gTg[NG + 1];
      gTg[0] = 0.0;
      for (int j = 1; j <= NG; ++j) gTg[j] = G(LT, kt + j);
      for (int j = NG; j >= 1; --j) {
        gR += G(LR, kt + j);
        const double Ta = exp(lT0[(kt + j - 1) * sp]), Tb = exp(lT0[(kt + j) * sp]);
        const double c = -2.0 * p.g_z * p.dz_hi[j - 1] / (p.R * (Ta + Tb) * (Ta + Tb));
        gTg[j - 1] += c * Ta * gR;
        gTg[j] += c * Tb * gR;
      }
      X(LR, kt) += gR;
      X(LT, kt) += gTg[0];
      for (int j = 1; j <= NG; ++j) X(LT, kt - j) += gTg[j];
    }
  }
}

__global__ __launch_bounds__(256) void k_fold_periodic(const KParams p, const double* __restrict__ Gb,
                                double* __restrict__ Xb) {
  const long long sp = p.splane;
  const long long n = (long long)NF * sp;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = int(i / sp);
    const long long col = i - (long long)f * sp;
    const double* G = Gb + f * p.sfield + col;
    double* X = Xb + f * p.sfield + col;
    for (int kz = NG; kz < NG + p.nz; ++kz) X[kz * sp] += G[kz * sp];
    for (int j = 0; j < NG; ++j) {
      X[(p.nz + j) * sp] += G[j * sp];              // below <- top of the interior
      X[(NG + j) * sp] += G[(p.nz + NG + j) * sp];  // above <- bottom of the interior
    }
  }
}

// Fourier part of the transpose: the filters are real, even multipliers, so
// each M_j = F^-1 diag(H_j) F is symmetric and Abar(0) += sum_j M_j Gbar(-j)
// (likewise at the top).  Planes: q = 0 Ax+iAy bottom, 1 Az bottom, 2 Ax+iAy
// top, 3 Az top; S[q*3 + j-1] holds Gbar of ghost j.
__global__ __launch_bounds__(256) void k_pack_ghost_cotangents(const KParams p, const double* __restrict__ Gb,
                                        double2* __restrict__ S) {
  const long long sp = p.splane;
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < sp;
       col += (long long)gridDim.x * blockDim.x) {
    for (int j = 1; j <= NG; ++j) {
      const long long ob = (NG - j) * sp + col, ot = (NG + p.nz - 1 + j) * sp + col;
      S[(0 * NG + j - 1) * sp + col] = make_double2(Gb[AX * p.sfield + ob], Gb[AY * p.sfield + ob]);
      S[(1 * NG + j - 1) * sp + col] = make_double2(Gb[AZ * p.sfield + ob], 0.0);
      S[(2 * NG + j - 1) * sp + col] = make_double2(Gb[AX * p.sfield + ot], Gb[AY * p.sfield + ot]);
      S[(3 * NG + j - 1) * sp + col] = make_double2(Gb[AZ * p.sfield + ot], 0.0);
    }
  }
}
__global__ __launch_bounds__(256) void k_pf_filter_T(const KParams p, const double2* __restrict__ S,
                              double2* __restrict__ T) {
  const long long sp = p.splane;
  const double inv_n = 1.0 / double(sp);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < 4 * sp;
       i += (long long)gridDim.x * blockDim.x) {
    const int q = int(i / sp);
    const long long col = i - q * sp;
    const int iy = int(col / p.nx), ix = int(col - (long long)iy * p.nx);
    const double k = kabs(p, ix, iy);
    const double* dist = p.pf_dist[q < 2 ? 0 : 1];
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 1; j <= NG; ++j) {
      const double fac = exp(-k * dist[j - 1]) * inv_n;
      const double2 v = S[(q * NG + j - 1) * sp + col];
      acc.x += v.x * fac;
      acc.y += v.y * fac;
    }
    T[i] = acc;
  }
}
__global__ __launch_bounds__(256) void k_unpack_fold_A(const KParams p, const double2* __restrict__ T,
                                double* __restrict__ Xb) {
  const long long sp = p.splane;
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < sp;
       col += (long long)gridDim.x * blockDim.x) {
    const long long ob = NG * sp + col, ot = (NG + p.nz - 1) * sp + col;
    Xb[AX * p.sfield + ob] += T[col].x;
    Xb[AY * p.sfield + ob] += T[col].y;
    Xb[AZ * p.sfield + ob] += T[sp + col].x;
    Xb[AX * p.sfield + ot] += T[2 * sp + col].x;
    Xb[AY * p.sfield + ot] += T[2 * sp + col].y;
    Xb[AZ * p.sfield + ot] += T[3 * sp + col].x;
  }
}

// ---------------------------------------------------------------------------
// element-wise pieces of the Runge-Kutta tangent and adjoint
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_state(const KParams& p, int f, int kz) {
  if (kz >= NG && kz < NG + p.nz) return true;
  return p.solar && kz < NG && (f == UX || f == UY);
}
__device__ __forceinline__ bool is_fixed(const KParams& p, int f, int kz) {
  if (!p.solar) return false;
  return (f == UZ && (kz == NG || kz == NG + p.nz - 1)) || (f == LR && kz == NG);
}

// dDF = P(alpha dDF + dt dR); dX = P(dX + beta dDF) over the state entries
__global__ __launch_bounds__(256) void k_tlm_combine(const KParams p, double alpha, double beta, double dt,
                              const double* __restrict__ dR, double* __restrict__ dDF,
                              double* __restrict__ dX) {
  const long long n = (long long)NF * p.sfield;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = int(i / p.sfield);
    const int kz = int((i - f * p.sfield) / p.splane);
    if (!is_state(p, f, kz)) continue;
    if (is_fixed(p, f, kz)) {
      dDF[i] = 0.0;
      dX[i] = 0.0;
      continue;
    }
    const double d = alpha * dDF[i] + dt * dR[i];
    dDF[i] = d;
    dX[i] = dX[i] + beta * d;
  }
}

// Xb = P Xb; dFb = P(dFb + beta Xb); Rb = dt dFb; dFb = alpha dFb
__global__ __launch_bounds__(256) void k_adj_combine(const KParams p, double alpha, double beta, double dt,
                              double* __restrict__ Xb, double* __restrict__ dFb,
                              double* __restrict__ Rb) {
  const long long n = (long long)NF * p.sfield;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = int(i / p.sfield);
    const int kz = int((i - f * p.sfield) / p.splane);
    if (!is_state(p, f, kz)) {
      Xb[i] = 0.0;
      dFb[i] = 0.0;
      Rb[i] = 0.0;
      continue;
    }
    if (is_fixed(p, f, kz)) {
      Xb[i] = 0.0;
      dFb[i] = 0.0;
      Rb[i] = 0.0;
      continue;
    }
    const double d = dFb[i] + beta * Xb[i];
    Rb[i] = dt * d;
    dFb[i] = alpha * d;
  }
}

// copy the state entries of src into dst and zero every other entry
__global__ __launch_bounds__(256) void k_copy_state_entries(const KParams p, const double* __restrict__ src,
                                     double* __restrict__ dst) {
  const long long n = (long long)NF * p.sfield;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = int(i / p.sfield);
    const int kz = int((i - f * p.sfield) / p.splane);
    dst[i] = is_state(p, f, kz) ? src[i] : 0.0;
  }
}

// adjoint of B_z on the plane at height z (linear between planes k0, k0+1)
__global__ __launch_bounds__(256) void k_bz_plane_vjp(const KParams p, int k0, double a, const double* __restrict__ bzb,
                               double* __restrict__ Xb) {
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < p.splane;
       col += (long long)gridDim.x * blockDim.x) {
    const int y = int(col / p.nx), x = int(col - (long long)y * p.nx);
    // d/dA_y of D1_x is -D1_x^T... : Abar_y += -D1_x(bzbar), Abar_x += +D1_y(bzbar)
    double dxb = 0.0, dyb = 0.0;
    for (int m = 1; m <= 3; ++m) {
      dxb += W1[m - 1] * (bzb[(long long)y * p.nx + wrapi(x + m, p.nx)] -
                          bzb[(long long)y * p.nx + wrapi(x - m, p.nx)]);
      dyb += W1[m - 1] * (bzb[(long long)wrapi(y + m, p.ny) * p.nx + x] -
                          bzb[(long long)wrapi(y - m, p.ny) * p.nx + x]);
    }
    dxb *= p.i60dx;
    dyb *= p.i60dy;
    for (int q = 0; q < 2; ++q) {
      const double wq = q == 0 ? 1.0 - a : a;
      if (wq == 0.0) continue;
      const long long o = (long long)(k0 + q + NG) * p.splane + col;
      Xb[AY * p.sfield + o] += -wq * dxb;
      Xb[AX * p.sfield + o] += wq * dyb;
    }
  }
}

int grid_of(long long n, int tpb) {
  long long b = (n + tpb - 1) / tpb;
  return int(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

}  // namespace

hipError_t launch_point_q(const KParams& p, const double* g, double* Q, hipStream_t s) {
  const long long n = (long long)p.nz * p.splane;
  hipLaunchKernelGGL(k_point_q, dim3(grid_of(n, 128)), dim3(128), 0, s, p, g, Q);
  return hipGetLastError();
}
hipError_t launch_point_jvp(const KParams& p, const double* Q, const double* dQ, const double* uh,
                            const double* ah, const double* duh, double ramp, double* dR,
                            hipStream_t s) {
  const long long n = (long long)p.nz * p.splane;
  hipLaunchKernelGGL(k_point_jvp, dim3(grid_of(n, 128)), dim3(128), 0, s, p, Q, dQ, uh, ah, duh,
                     ramp, dR);
  return hipGetLastError();
}
hipError_t launch_ghost_rows_jvp(const KParams& p, const double* dX, const double* duh,
                                 double ramp, double* dR, hipStream_t s) {
  hipLaunchKernelGGL(k_ghost_rows_jvp, dim3(grid_of(2LL * NG * p.splane, 256)), dim3(256), 0, s, p,
                     dX, duh, ramp, dR);
  return hipGetLastError();
}
hipError_t launch_point_vjp(const KParams& p, const double* Q, const double* Rbar,
                            const double* uh, const double* ah, double ramp, double* Qbar,
                            double* uhbar, hipStream_t s) {
  const long long n = (long long)p.nz * p.splane;
  hipLaunchKernelGGL(k_point_vjp, dim3(grid_of(n, 128)), dim3(128), 0, s, p, Q, Rbar, uh, ah, ramp,
                     Qbar, uhbar);
  return hipGetLastError();
}
hipError_t launch_ghost_rows_vjp(const KParams& p, const double* Rbar, double ramp, double* Xbar,
                                 double* uhbar, hipStream_t s) {
  hipLaunchKernelGGL(k_ghost_rows_vjp, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p, Rbar, ramp,
                     Xbar, uhbar);
  return hipGetLastError();
}
hipError_t launch_stencil_T(const KParams& p, const double* Qbar, double* Gbar, hipStream_t s) {
  const long long n = (long long)(p.nz + 2 * NG) * p.splane;
  hipLaunchKernelGGL(k_stencil_T, dim3(grid_of(n, 128)), dim3(128), 0, s, p, Qbar, Gbar);
  return hipGetLastError();
}
hipError_t launch_fill_lin(const KParams& p, const double* g, double* dg, double2* scratch,
                           hipStream_t s) {
  if (!p.solar) return launch_fill_periodic_z(p, dg, s);
  hipLaunchKernelGGL(k_fill_solar_columns_lin, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p, g,
                     dg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_potential_ghosts(p, dg, scratch, s);   // linear in A
}
hipError_t launch_fold_ghosts_T(const KParams& p, const double* g, const double* Gbar,
                                double* Xbar, double2* scratch, hipStream_t s) {
  if (!p.solar) {
    hipLaunchKernelGGL(k_fold_periodic, dim3(grid_of((long long)NF * p.splane, 256)), dim3(256), 0,
                       s, p, Gbar, Xbar);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_fold_solar, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p, g, Gbar, Xbar);
  double2* S = scratch;                    // 12 planes
  double2* T = scratch + 12 * p.splane;    // 4 planes
  hipLaunchKernelGGL(k_pack_ghost_cotangents, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p,
                     Gbar, S);
  hipError_t e = fft2d(p, S, 12, -1.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pf_filter_T, dim3(grid_of(4 * p.splane, 256)), dim3(256), 0, s, p, S, T);
  e = fft2d(p, T, 4, +1.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack_fold_A, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p, T, Xbar);
  return hipGetLastError();
}
hipError_t launch_tlm_combine(const KParams& p, double alpha, double beta, double dt,
                              const double* dR, double* dDF, double* dX, hipStream_t s) {
  hipLaunchKernelGGL(k_tlm_combine, dim3(grid_of((long long)NF * p.sfield, 256)), dim3(256), 0, s,
                     p, alpha, beta, dt, dR, dDF, dX);
  return hipGetLastError();
}
hipError_t launch_adj_combine(const KParams& p, double alpha, double beta, double dt, double* Xb,
                              double* dFb, double* Rb, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_combine, dim3(grid_of((long long)NF * p.sfield, 256)), dim3(256), 0, s,
                     p, alpha, beta, dt, Xb, dFb, Rb);
  return hipGetLastError();
}
hipError_t launch_copy_state_entries(const KParams& p, const double* src, double* dst,
                                     hipStream_t s) {
  hipLaunchKernelGGL(k_copy_state_entries, dim3(grid_of((long long)NF * p.sfield, 256)), dim3(256),
                     0, s, p, src, dst);
  return hipGetLastError();
}
hipError_t launch_bz_plane_vjp_k(const KParams& p, int k0, double a, const double* bzbar,
                                 double* Xbar, hipStream_t s) {
  hipLaunchKernelGGL(k_bz_plane_vjp, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p, k0, a, bzbar,
                     Xbar);
  return hipGetLastError();
}
hipError_t launch_bz_plane_vjp(const KParams& p, double zq, const double* bzbar, double* Xbar,
                               hipStream_t s) {
  const double kf = (zq - p.z0) / p.dz;
  int k0 = int(floor(kf));
  double a = kf - k0;
  if (k0 >= p.nz - 1) {
    k0 = p.nz - 2;
    a = 1.0;
  }
  hipLaunchKernelGGL(k_bz_plane_vjp, dim3(grid_of(p.splane, 256)), dim3(256), 0, s, p, k0, a, bzbar,
                     Xbar);
  return hipGetLastError();
}

}  // namespace cmhd
