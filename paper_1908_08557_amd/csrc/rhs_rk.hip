// Fused substage kernel: sixth-order stencils + pointwise right-hand side +
// 2N-RK3 register update, one thread per (x, y) column of a 16 x 16 tile,
// marching in z over a chunk of planes.
//
// Per plane k the block stages into LDS, for the 22 x 22 haloed tile
// (x, y periodic by index wrap):
//   P[f]  the values of the 8 fields at plane k (float64), and
//   Zs[f] d/dz of A, u, ln T at plane k (7 fields),
// so that every x/y derivative, the xy mixed derivatives (D1_y D1_x, the
// 36-point product stencil) and the xz/yz mixed derivatives (D1_x and D1_y
// of the staged d/dz) come from LDS.  The pure z derivatives of the own
// column stay in registers.  Then
//   dF <- alpha dF + dt RHS,   f_next <- f + beta dF
// is applied in float64 and written once.
#include "cmhd_internal.h"
#include "rhs_point.h"

namespace cmhd {
namespace {

// unscaled sixth-order stencils: 60 h D1 and 180 h^2 D2 at index c, stride s
template <typename R>
__device__ __forceinline__ R d1u(const R* a, int c, int s) {
  return R(45.0) * (a[c + s] - a[c - s]) - R(9.0) * (a[c + 2 * s] - a[c - 2 * s]) +
         (a[c + 3 * s] - a[c - 3 * s]);
}
__device__ __forceinline__ double d2u(const double* a, int c, int s) {
  return -490.0 * a[c] + 270.0 * (a[c + s] + a[c - s]) - 27.0 * (a[c + 2 * s] + a[c - 2 * s]) +
         2.0 * (a[c + 3 * s] + a[c - 3 * s]);
}
// 3600 h_x h_y d_x d_y: D1 along y of D1 along x (product stencil)
__device__ __forceinline__ double dxyu(const double* a, int c) {
  return 45.0 * (d1u(a, c + HX, 1) - d1u(a, c - HX, 1)) -
         9.0 * (d1u(a, c + 2 * HX, 1) - d1u(a, c - 2 * HX, 1)) +
         (d1u(a, c + 3 * HX, 1) - d1u(a, c - 3 * HX, 1));
}


// Derivatives at the own column, read from the staged plane on demand.
template <typename Real>
struct LdsSource {
  static constexpr int kUnroll = 1;   // rolled component loops
  const double (*P)[HP];
  const Real (*Zs)[HP];
  const double (*D2z)[NT];
  int c, t;
  double i60dx, i60dy, i180dx2, i180dy2;
  __device__ __forceinline__ Real v(int f) const { return Real(P[f][c]); }
  __device__ __forceinline__ double v64(int f) const { return P[f][c]; }
  __device__ __forceinline__ Real d(int f, int dir) const {
    if (dir == 0) return Real(d1u(P[f], c, 1) * i60dx);
    if (dir == 1) return Real(d1u(P[f], c, HX) * i60dy);
    return Zs[f][c];
  }
  __device__ __forceinline__ Real h(int f, int slot) const {
    switch (slot) {
      case 0: return Real(d2u(P[f], c, 1) * i180dx2);
      case 1: return Real(d2u(P[f], c, HX) * i180dy2);
      case 2: return Real(D2z[f][t]);
      case 3: return Real(dxyu(P[f], c) * (i60dx * i60dy));
      case 4: return d1u(Zs[f], c, 1) * Real(i60dx);
      default: return d1u(Zs[f], c, HX) * Real(i60dy);
    }
  }
  __device__ __forceinline__ Real lapr() const {
    return Real(d2u(P[LR], c, 1) * i180dx2 + d2u(P[LR], c, HX) * i180dy2 + D2z[LR][t]);
  }
};

__device__ __forceinline__ void swamp(const KParams& p, int k, double& w, double& dw) {
  w = 0.0;
  dw = 0.0;
  if (!p.solar || (p.eta_s == 0.0 && p.chi_s == 0.0 && p.chi_rho == 0.0)) return;
  const double z = p.z0 + k * p.dz;
  const double L = p.z_t - p.z_s;
  double s = (z - p.z_s) / L;
  s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  w = s * s * (3.0 - 2.0 * s);
  dw = (z > p.z_s && z < p.z_t) ? 6.0 * s * (1.0 - s) / L : 0.0;
}

template <typename Real, bool SOLAR, bool READ_DF, bool WRITE_DF>
__global__ __launch_bounds__(NT) void k_rhs_rk(const double* __restrict__ f,
                                               double* __restrict__ fo,
                                               double* __restrict__ dF,
                                               const double* __restrict__ uh,
                                               const double* __restrict__ ah, const KParams p,
                                               const StageArgs st, int kchunk) {
  __shared__ double P[NF][HP];
  __shared__ Real Zs[NF][HP];     // d/dz (the ln rho slot only at the tile's own columns)
  __shared__ double D2z[NF][NT];  // d2/dz2 at the tile's own columns

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const long long sp = p.splane, sf = p.sfield;
  const long long col = (long long)(y0 + ty) * p.nx + (x0 + tx);
  const int c = (ty + NG) * HX + (tx + NG);

  // the halo column this thread stages (threads 0 .. NHALO-1)
  int hc = -1;
  long long hcol = 0;
  if (tid < NHALO) {
    int r, q;
    if (tid < 2 * NG * HX) {
      const int row = tid / HX;
      r = row < NG ? row : row + TY;
      q = tid % HX;
    } else {
      const int j = tid - 2 * NG * HX;
      r = NG + j / (2 * NG);
      const int c6 = j % (2 * NG);
      q = c6 < NG ? c6 : c6 + TX;
    }
    hc = r * HX + q;
    int gx = x0 + q - NG, gy = y0 + r - NG;
    gx += gx < 0 ? p.nx : 0;
    gx -= gx >= p.nx ? p.nx : 0;
    gy += gy < 0 ? p.ny : 0;
    gy -= gy >= p.ny ? p.ny : 0;
    hcol = (long long)gy * p.nx + gx;
  }

  const int oc = int(col), oh = int(hcol), sp32 = int(sp);
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(kbeg + kchunk, p.nz);
  for (int k = kbeg; k < kend; ++k) {
    const long long zo = (long long)(k + NG) * sp;

    // ---- stage plane k: own column (values, d/dz, d2/dz2) and one halo column.
    // Addresses: a wave-uniform base at plane k-3 per field plus non-negative
    // 32-bit per-thread offsets (no 64-bit pointer per field and plane).
    const long long zb = (long long)k * sp;   // plane k-3 in array planes
    // one field at a time (rolled loop: keeps the loads in flight, and so the
    // registers, bounded)
#pragma unroll 1
    for (int fi = 0; fi < NF; ++fi) {
      const double* __restrict__ fb = f + (fi * sf + zb);
      const double m3 = fb[oc], m2 = fb[oc + sp32], m1 = fb[oc + 2 * sp32];
      const double c0 = fb[oc + 3 * sp32];
      const double p1 = fb[oc + 4 * sp32], p2 = fb[oc + 5 * sp32], p3 = fb[oc + 6 * sp32];
      P[fi][c] = c0;
      Zs[fi][c] = Real((45.0 * (p1 - m1) - 9.0 * (p2 - m2) + (p3 - m3)) * p.i60dz);
      D2z[fi][tid] = (-490.0 * c0 + 270.0 * (p1 + m1) - 27.0 * (p2 + m2) + 2.0 * (p3 + m3)) *
                     p.i180dz2;
      if (hc >= 0) {
        P[fi][hc] = fb[oh + 3 * sp32];
        if (fi != LR) {
          const double d1 = (45.0 * (fb[oh + 4 * sp32] - fb[oh + 2 * sp32]) -
                             9.0 * (fb[oh + 5 * sp32] - fb[oh + sp32]) +
                             (fb[oh + 6 * sp32] - fb[oh])) *
                            p.i60dz;
          Zs[fi][hc] = Real(d1);
        }
      }
    }
    __syncthreads();

    // ---- pointwise right-hand side, derivatives read from LDS on demand
    LdsSource<Real> src{P, Zs, D2z, c, tid, p.i60dx, p.i60dy, p.i180dx2, p.i180dy2};
    PointCtx<Real> pc;
    swamp(p, k, pc.w, pc.dw);
    pc.bottom = SOLAR && k == 0;
    pc.top = SOLAR && k == p.nz - 1;
    pc.ramp = st.ramp;
    if (SOLAR && k == 0) {
      pc.uh[0] = Real(uh[oc]);
      pc.uh[1] = Real(uh[sp + oc]);
      pc.ah[0] = Real(ah[oc]);
      pc.ah[1] = Real(ah[sp + oc]);
    } else {
      pc.uh[0] = pc.uh[1] = pc.ah[0] = pc.ah[1] = Real(0.0);
    }

    Real out[NF];
    rhs_eval<Real>(src, pc, p, out);

    // ---- 2N-RK3 register update in float64
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const long long fo_off = fi * sf + zo;
      const double r = double(out[fi]);
      double d = READ_DF ? st.alpha * dF[fo_off + oc] + st.dt * r : st.dt * r;
      double fn = P[fi][c] + st.beta * d;
      if (SOLAR) {
        // closed boundary (u_z = 0 at both boundary planes) and the
        // photospheric density held at its initial value ('fg')
        const bool fixz = (fi == UZ) && (k == 0 || k == p.nz - 1);
        const bool fixr = (fi == LR) && (k == 0);
        if (fixz || fixr) {
          d = 0.0;
          fn = fixr ? p.lnrho0_bot[3] : 0.0;
        }
      }
      if (WRITE_DF) dF[fo_off + oc] = d;
      fo[fo_off + oc] = fn;
    }
    __syncthreads();
  }
}

// The u_x, u_y rows of the three lower ghost planes evolve under the nudging
// term alone (eq. 5: never imposed directly).
__global__ void k_ghost_rows(const double* __restrict__ f, double* __restrict__ fo,
                             double* __restrict__ dF, const double* __restrict__ uh,
                             const KParams p, const StageArgs st, int read_dF, int write_dF) {
  const long long n = 2LL * NG * p.splane;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int comp = int(i / (NG * p.splane));
    const long long rem = i - comp * NG * p.splane;   // plane j (k = j-3) and column
    const long long col = rem % p.splane;
    const long long idx = (UX + comp) * p.sfield + rem;
    const double r = -p.tau_u * (f[idx] - st.ramp * uh[comp * p.splane + col]);
    const double d = read_dF ? st.alpha * dF[idx] + st.dt * r : st.dt * r;
    if (write_dF) dF[idx] = d;
    fo[idx] = f[idx] + st.beta * d;
  }
}

template <typename Real, bool SOLAR>
hipError_t launch_typed(const KParams& p, int stage, const double* f, double* fo, double* dF,
                        const double* uh, const double* ah, StageArgs st, hipStream_t s) {
  const int tiles = (p.nx / TX) * (p.ny / TY);
  int nchunk = (2048 + tiles - 1) / tiles;
  if (nchunk > p.nz) nchunk = p.nz;
  const int kchunk = (p.nz + nchunk - 1) / nchunk;
  nchunk = (p.nz + kchunk - 1) / kchunk;
  dim3 grid(p.nx / TX, p.ny / TY, nchunk);
  if (stage == 0)
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, false, true>), grid, dim3(NT), 0, s, f, fo, dF, uh,
                       ah, p, st, kchunk);
  else if (stage == 1)
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, true, true>), grid, dim3(NT), 0, s, f, fo, dF, uh,
                       ah, p, st, kchunk);
  else
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, true, false>), grid, dim3(NT), 0, s, f, fo, dF, uh,
                       ah, p, st, kchunk);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs_rk(const KParams& p, int prec, int stage, const double* f, double* fo,
                         double* dF, const double* uh, const double* ah, StageArgs st,
                         hipStream_t s) {
  if (prec == CMHD_FP32_SPLIT)
    return p.solar ? launch_typed<float, true>(p, stage, f, fo, dF, uh, ah, st, s)
                   : launch_typed<float, false>(p, stage, f, fo, dF, uh, ah, st, s);
  return p.solar ? launch_typed<double, true>(p, stage, f, fo, dF, uh, ah, st, s)
                 : launch_typed<double, false>(p, stage, f, fo, dF, uh, ah, st, s);
}

hipError_t launch_ghost_rows(const KParams& p, const double* f, double* fo, double* dF,
                             const double* uh, StageArgs st, int read_dF, int write_dF,
                             hipStream_t s) {
  const long long n = 2LL * NG * p.splane;
  const int blocks = int((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_ghost_rows, dim3(blocks), dim3(256), 0, s, f, fo, dF, uh, p, st, read_dF,
                     write_dF);
  return hipGetLastError();
}

}  // namespace cmhd
