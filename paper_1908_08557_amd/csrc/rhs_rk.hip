// One 2N-RK3 substage in two kernels.
//
// k_zderiv streams the state once in z and writes the sixth-order d/dz and
// d2/dz2 of the 8 fields (16 slots, [slot][nz][ny][nx], in the precision of
// the right-hand side).
//
// k_rhs_rk: one thread per (x, y) column of a 16 x 16 tile, marching in z.
// Every input it needs at plane k is single-plane data, so plane k+1 is
// staged into LDS by direct global->LDS copies (16-byte lanes, no registers
// in flight) while plane k is being computed:
//   P   the 8 fields on the 22 x 24 haloed plane (x0-4 .. x0+19, y0-3 .. y0+18)
//   Zs  d/dz of A, u, ln T on the same haloed plane (for the xz, yz mixed
//       derivatives D1_x D1_z, D1_y D1_z)
//   Zo  d/dz ln rho and the 8 d2/dz2 at the own columns
//   DF  the RK register at the own columns (substages 2 and 3)
// Per plane:
//   1a  stencils from LDS -> the 72 pointwise inputs q in registers; D1_x of
//       the six fields with an xy mixed derivative on the tile and its y halo
//       -> LDS
//   --  barrier; the copies of plane k+1 (and the RK register of plane k) are
//       issued
//   1b  xy mixed derivatives D1_y (D1_x f) from LDS
//   2   pointwise right-hand side from registers (rhs_eval)
//   --  wait for the copies, barrier
//   3   dF <- alpha dF + dt RHS, f_next <- f + beta dF in float64, stored once
// The arithmetic of every derivative is that of the product stencils applied
// to the float64 state (differences formed in float64, then rounded to the
// precision of the right-hand side).
#include "cmhd_internal.h"
#include "qslots.h"
#include "rhs_point.h"

namespace cmhd {
namespace {

// haloed plane: RW x RH, x from x0-4 (16-byte aligned rows), y from y0-3
constexpr int RW = 24, RH = 22, RPL = RW * RH;
constexpr int DXW = TX, DXH = RH;   // D1_x on the tile columns and all 22 rows
constexpr int NZS = 7;              // haloed d/dz: A_x A_y A_z u_x u_y u_z ln T
constexpr int NZO = 9;              // own d/dz ln rho, then d2/dz2 of the 8 fields
constexpr int NDX = 6;              // xy mixed: A_x A_y A_z u_x u_y ln T
constexpr int NZSLOT = 2 * NF;      // slots of the z-derivative buffer

__device__ __forceinline__ constexpr int zs_index(int f) { return f < LR ? f : (f == LT ? 6 : -1); }
__device__ __forceinline__ constexpr int dx_index(int f) { return f <= UY ? f : (f == LT ? 5 : -1); }

template <typename Real>
struct Stage {
  double P[NF][RPL];
  Real Zs[NZS][RPL];
  Real Zo[NZO][NT];
  double Dx[NDX][DXH * DXW];
  double DF[NF][NT];
};

template <typename T>
using lds = __attribute__((address_space(3))) T;

// An LDS pointer the compiler cannot see through, re-made at every plane:
// every access is then this base plus a small non-negative immediate, and no
// per-offset addresses are precomputed and held across the plane loop.
template <typename T>
__device__ __forceinline__ lds<T>* lds_base(T* p) {
  lds<T>* q = (lds<T>*)p;
  asm volatile("" : "+v"(q));
  return q;
}

// unscaled sixth-order D1 (60 h D1) at index c, stride s
template <typename Ptr>
__device__ __forceinline__ auto d1u(Ptr a, int c, int s) {
  using R = typename std::remove_cv<typename std::remove_reference<decltype(a[0])>::type>::type;
  return R(45.0) * (a[c + s] - a[c - s]) - R(9.0) * (a[c + 2 * s] - a[c - 2 * s]) +
         (a[c + 3 * s] - a[c - 3 * s]);
}

// one 16-byte global->LDS copy per lane: lane l of the wave writes
// lds_base + 16 l (the destination is wave-uniform)
__device__ __forceinline__ void copy16(const void* gsrc, void* lds_base) {
  __builtin_amdgcn_global_load_lds(gsrc, (__attribute__((address_space(3))) void*)lds_base, 16,
                                   0, 0);
}

// Lane offsets (bytes, relative to the (slot, plane) base) of the 16-byte
// chunks of a region, elements of E bytes.  Chunk m*64 + lane of the haloed
// plane (RH rows of RW elements, x0-4 / y0-3 origin, periodic wrap) or of the
// own 16 x 16 tile.  Chunks never straddle the periodic seam: x origins are
// multiples of 16/E and nx is a multiple of 16.
template <int E>
struct Chunks {
  static constexpr int K = 16 / E;
  static constexpr int HCR = RW / K, HN = RH * HCR, HI = (HN + 63) / 64;
  static constexpr int OCR = TX / K, ON = TY * OCR, OI = (ON + 63) / 64;
  static __device__ unsigned halo(int m, int lane, int x0, int y0, int nx, int ny) {
    int ch = m * 64 + lane;
    ch = ch < HN ? ch : 0;
    const int row = ch / HCR, cc = ch - row * HCR;
    int x = x0 - 4 + cc * K, y = y0 - NG + row;
    x += x < 0 ? nx : 0;
    x -= x >= nx ? nx : 0;
    y += y < 0 ? ny : 0;
    y -= y >= ny ? ny : 0;
    return unsigned((y * nx + x) * E);
  }
  static __device__ unsigned own(int m, int lane, int x0, int y0, int nx) {
    int ch = m * 64 + lane;
    ch = ch < ON ? ch : 0;
    const int row = ch / OCR, cc = ch - row * OCR;
    return unsigned(((y0 + row) * nx + x0 + cc * K) * E);
  }
};
static_assert(Chunks<8>::HI == 5 && Chunks<8>::OI == 2 && Chunks<4>::HI == 3 &&
                  Chunks<4>::OI == 1, "chunk counts");

// this wave's share of the copies of one plane: wave w issues the chunk
// groups m = w, w+4, ... of every array
template <typename Real>
struct Copier {
  using CD = Chunks<8>;
  using CR = Chunks<sizeof(Real)>;
  unsigned hd[2], hr[2], od, orl;   // lane offsets of the wave's groups
  int w, lane;
  __device__ void init(int w_, int lane_, int x0, int y0, int nx, int ny) {
    w = w_;
    lane = lane_;
    hd[0] = CD::halo(w, lane, x0, y0, nx, ny);
    hd[1] = CD::halo(w + 4, lane, x0, y0, nx, ny);
    hr[0] = CR::halo(w, lane, x0, y0, nx, ny);
    hr[1] = CR::halo(w + 4, lane, x0, y0, nx, ny);
    od = CD::own(w, lane, x0, y0, nx);
    orl = CR::own(w, lane, x0, y0, nx);
  }
  template <int E>
  __device__ void halo_group(const char* base, char* lds, int m, unsigned off) const {
    using C = Chunks<E>;
    if (m < C::HI && m * 64 + lane < C::HN) copy16(base + off, lds + m * 1024);
  }
  template <int E>
  __device__ void own_group(const char* base, char* lds, int m, unsigned off) const {
    using C = Chunks<E>;
    if (m < C::OI && m * 64 + lane < C::ON) copy16(base + off, lds + m * 1024);
  }
  // the plane-k inputs: state (array plane k+NG) and z derivatives (plane k)
  __device__ void plane(Stage<Real>& S, const double* f, const Real* dz, long long sf,
                        long long sp, long long szs, int k) const {
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const char* b = reinterpret_cast<const char*>(f + fi * sf + (k + NG) * sp);
      halo_group<8>(b, reinterpret_cast<char*>(S.P[fi]), w, hd[0]);
      halo_group<8>(b, reinterpret_cast<char*>(S.P[fi]), w + 4, hd[1]);
    }
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      if (fi == LR) continue;
      const char* b = reinterpret_cast<const char*>(dz + fi * szs + k * sp);
      halo_group<sizeof(Real)>(b, reinterpret_cast<char*>(S.Zs[zs_index(fi)]), w, hr[0]);
      halo_group<sizeof(Real)>(b, reinterpret_cast<char*>(S.Zs[zs_index(fi)]), w + 4, hr[1]);
    }
#pragma unroll
    for (int s = 0; s < NZO; ++s) {
      const int slot = s == 0 ? LR : NF + (s - 1);
      const char* b = reinterpret_cast<const char*>(dz + slot * szs + k * sp);
      own_group<sizeof(Real)>(b, reinterpret_cast<char*>(S.Zo[s]), w, orl);
    }
  }
  __device__ void rk_register(Stage<Real>& S, const double* dF, long long sf, long long sp,
                              int k) const {
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const char* b = reinterpret_cast<const char*>(dF + fi * sf + (k + NG) * sp);
      own_group<8>(b, reinterpret_cast<char*>(S.DF[fi]), w, od);
    }
  }
};

// Source for rhs_eval: the derivatives of A are read from the staged plane on
// demand (rolled component loop, few registers), everything else from the
// inputs gathered into registers (indices are compile-time constants).
constexpr int PC = NG * RW + NG;   // own point relative to a haloed-plane base
constexpr int DC = NG * DXW;       // own point relative to the D1_x base

template <typename Real>
struct HybridSource {
  static constexpr int kUnrollA = 1, kUnrollU = 3;
  const Real* q;
  const double* v64s;
  lds<double>* pP;
  lds<Real>* pZ;
  lds<Real>* pO;
  lds<double>* pD;
  double i60dx, i60dy, i180dx2, i180dy2, ixy;
  __device__ __forceinline__ Real v(int f) const { return q[q_v(f)]; }
  __device__ __forceinline__ double v64(int f) const { return v64s[f]; }
  __device__ __forceinline__ Real d(int f, int dir) const {
    if (f <= AZ && dir == 1) return Real(d1u(pP, f * RPL + PC, RW) * i60dy);
    if (f <= AZ && dir == 2) return pZ[f * RPL + PC];
    return q[q_d(f, dir)];
  }
  __device__ __forceinline__ Real h(int f, int s) const {
    if (f <= AZ) {
      const int b = f * RPL + PC;
      switch (s) {
        case 0: {
          const double c0 = pP[b];
          return Real((-490.0 * c0 + 270.0 * (pP[b + 1] + pP[b - 1]) -
                       27.0 * (pP[b + 2] + pP[b - 2]) + 2.0 * (pP[b + 3] + pP[b - 3])) *
                      i180dx2);
        }
        case 1: {
          const double c0 = pP[b];
          return Real((-490.0 * c0 + 270.0 * (pP[b + RW] + pP[b - RW]) -
                       27.0 * (pP[b + 2 * RW] + pP[b - 2 * RW]) +
                       2.0 * (pP[b + 3 * RW] + pP[b - 3 * RW])) *
                      i180dy2);
        }
        case 2: return pO[(1 + f) * NT];
        case 3: return Real(d1u(pD, f * DXH * DXW + DC, DXW) * ixy);
        case 4: return d1u(pZ, b, 1) * Real(i60dx);
        default: return d1u(pZ, b, RW) * Real(i60dy);
      }
    }
    const int slot = q_h(f, s);
    return slot >= 0 ? q[slot] : Real(0.0);
  }
  __device__ __forceinline__ Real lapr() const { return q[Q_LAPR]; }
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

// ---------------------------------------------------------------------------
// z derivatives: one thread per (column, field), marching over a chunk of
// planes with the 7-plane window in registers
template <typename Real>
__global__ __launch_bounds__(256) void k_zderiv(const double* __restrict__ f,
                                                Real* __restrict__ dz, const KParams p,
                                                int kchunk) {
  const long long sp = p.splane;
  const long long col = blockIdx.x * 256LL + threadIdx.x;
  const int fi = blockIdx.y;
  const int k0 = blockIdx.z * kchunk;
  const int k1 = min(k0 + kchunk, p.nz);
  const long long szs = (long long)p.nz * sp;
  const double* a = f + fi * p.sfield + col;   // array plane j at a[j * sp]
  Real* o1 = dz + fi * szs + col;
  Real* o2 = dz + (NF + fi) * szs + col;
  double w0 = a[(k0 + 0) * sp], w1 = a[(k0 + 1) * sp], w2 = a[(k0 + 2) * sp];
  double w3 = a[(k0 + 3) * sp], w4 = a[(k0 + 4) * sp], w5 = a[(k0 + 5) * sp];
  for (int k = k0; k < k1; ++k) {
    const double w6 = a[(k + 6) * sp];
    const double d1 = (45.0 * (w4 - w2) - 9.0 * (w5 - w1) + (w6 - w0)) * p.i60dz;
    const double d2 = (-490.0 * w3 + 270.0 * (w4 + w2) - 27.0 * (w5 + w1) + 2.0 * (w6 + w0)) *
                      p.i180dz2;
    o1[k * sp] = Real(d1);
    o2[k * sp] = Real(d2);
    w0 = w1;
    w1 = w2;
    w2 = w3;
    w3 = w4;
    w4 = w5;
    w5 = w6;
  }
}

// ---------------------------------------------------------------------------
template <typename Real, bool SOLAR, bool READ_DF, bool WRITE_DF>
__global__ __launch_bounds__(NT) void k_rhs_rk(const double* __restrict__ f,
                                               const Real* __restrict__ dz,
                                               double* __restrict__ fo,
                                               double* __restrict__ dF,
                                               const double* __restrict__ uh,
                                               const double* __restrict__ ah, const KParams p,
                                               const StageArgs st, int kchunk) {
  __shared__ __align__(16) Stage<Real> S;
  constexpr bool kFloat = !std::is_same<Real, double>::value;

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const long long sp = p.splane, sf = p.sfield, szs = (long long)p.nz * sp;
  const int oc = (y0 + ty) * p.nx + (x0 + tx);    // own column within a plane
  const int c = (ty + NG) * RW + (tx + 4);        // own point in the haloed plane
  const int cx = (ty + NG) * DXW + tx;            // own point in the D1_x array

  Copier<Real> cp;
  cp.init(__builtin_amdgcn_readfirstlane(tid / 64), tid % 64, x0, y0, p.nx, p.ny);

  // y-halo rows of D1_x computed by threads 0..95: rows 0-2 and 19-21
  const int hrow = tid < 3 * TX ? tid / TX : TY + NG + (tid - 3 * TX) / TX;
  const int hcol = tid % TX;

  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(kbeg + kchunk, p.nz);

  cp.plane(S, f, dz, sf, sp, szs, kbeg);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int k = kbeg; k < kend; ++k) {
    // ---- 1a: stencils of the staged plane into registers (all but the
    // derivatives of A, which the magnetic part reads on demand); D1_x of the
    // xy-mixed fields into LDS.  Bases sit at the lowest address each array
    // is read at, so that all offsets are non-negative immediates.
    const auto pP = lds_base(&S.P[0][c - PC]);
    const auto pZ = lds_base(&S.Zs[0][c - PC]);
    const auto pO = lds_base(&S.Zo[0][tid]);
    const auto pD = lds_base(&S.Dx[0][cx - DC]);
    Real q[NQ];
    double v64[NF];
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const int b = fi * RPL + PC;
      const double c0 = pP[b];
      const double xm1 = pP[b - 1], xp1 = pP[b + 1], xm2 = pP[b - 2], xp2 = pP[b + 2];
      const double xm3 = pP[b - 3], xp3 = pP[b + 3];
      const double d1x = 45.0 * (xp1 - xm1) - 9.0 * (xp2 - xm2) + (xp3 - xm3);
      v64[fi] = c0;
      q[q_v(fi)] = Real(c0);
      q[q_d(fi, 0)] = Real(d1x * p.i60dx);
      if (dx_index(fi) >= 0) pD[dx_index(fi) * DXH * DXW + DC] = d1x;
      if (fi > AZ) {
        const double ym1 = pP[b - RW], yp1 = pP[b + RW], ym2 = pP[b - 2 * RW];
        const double yp2 = pP[b + 2 * RW], ym3 = pP[b - 3 * RW], yp3 = pP[b + 3 * RW];
        const double d1y = 45.0 * (yp1 - ym1) - 9.0 * (yp2 - ym2) + (yp3 - ym3);
        const double d2x =
            -490.0 * c0 + 270.0 * (xp1 + xm1) - 27.0 * (xp2 + xm2) + 2.0 * (xp3 + xm3);
        const double d2y =
            -490.0 * c0 + 270.0 * (yp1 + ym1) - 27.0 * (yp2 + ym2) + 2.0 * (yp3 + ym3);
        q[q_d(fi, 1)] = Real(d1y * p.i60dy);
        if (fi == LR) {
          q[q_d(fi, 2)] = pO[0];
          q[Q_LAPR] = Real(d2x * p.i180dx2 + d2y * p.i180dy2 + double(pO[(1 + LR) * NT]));
        } else {
          const int zb = zs_index(fi) * RPL + PC;
          q[q_d(fi, 2)] = pZ[zb];
          q[q_h(fi, 0)] = Real(d2x * p.i180dx2);
          q[q_h(fi, 1)] = Real(d2y * p.i180dy2);
          q[q_h(fi, 2)] = pO[(1 + fi) * NT];
          if (q_h(fi, 4) >= 0) q[q_h(fi, 4)] = d1u(pZ, zb, 1) * Real(p.i60dx);
          if (q_h(fi, 5) >= 0) q[q_h(fi, 5)] = d1u(pZ, zb, RW) * Real(p.i60dy);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // D1_x on the y-halo rows (threads 0..95)
    if (tid < 2 * NG * TX) {
      const auto pPh = lds_base(&S.P[0][hrow * RW + hcol + 4 - NG]);
      const auto pDh = lds_base(&S.Dx[0][hrow * DXW + hcol]);
#pragma unroll
      for (int fi = 0; fi < NF; ++fi)
        if (dx_index(fi) >= 0) pDh[dx_index(fi) * DXH * DXW] = d1u(pPh, fi * RPL + NG, 1);
    }
    __syncthreads();

    // ---- 1b: xy mixed derivatives D1_y (D1_x f) of u_x, u_y, ln T
    const double ixy = p.i60dx * p.i60dy;
#pragma unroll
    for (int fi = UX; fi < NF; ++fi)
      if (dx_index(fi) >= 0)
        q[q_h(fi, 3)] = Real(d1u(pD, dx_index(fi) * DXH * DXW + DC, DXW) * ixy);

    // ---- 2a: magnetic part of the right-hand side (A read from LDS)
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
    const HybridSource<Real> src{q,      v64,     pP,        pZ,        pO, pD,
                                 p.i60dx, p.i60dy, p.i180dx2, p.i180dy2, ixy};
    Real out[NF];
    MagState<Real> mag;
    rhs_magnetic<Real>(src, pc, p, out, mag);
    __syncthreads();

    // ---- copies: the RK register of this plane, then the next plane
    if (READ_DF) cp.rk_register(S, dF, sf, sp, k);
    if (k + 1 < kend) cp.plane(S, f, dz, sf, sp, szs, k + 1);

    // ---- 2b: fluid part of the right-hand side, from registers
    rhs_fluid<Real>(src, pc, p, mag, out);

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- 3: 2N-RK3 register update in float64
    const auto pF = lds_base(&S.DF[0][tid]);
    const unsigned ob = unsigned(oc) * 8u;   // byte offset of the own column
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const long long pl = fi * sf + (k + NG) * sp;   // uniform
      const double r = double(out[fi]);
      double d = READ_DF ? st.alpha * pF[fi * NT] + st.dt * r : st.dt * r;
      double fn = v64[fi] + st.beta * d;
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
      if (WRITE_DF) *reinterpret_cast<double*>(reinterpret_cast<char*>(dF + pl) + ob) = d;
      *reinterpret_cast<double*>(reinterpret_cast<char*>(fo + pl) + ob) = fn;
    }
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

int zchunks(const KParams& p, int target_blocks, int& kchunk) {
  const int tiles = (p.nx / TX) * (p.ny / TY);
  int nchunk = (target_blocks + tiles - 1) / tiles;
  if (nchunk > p.nz) nchunk = p.nz;
  kchunk = (p.nz + nchunk - 1) / nchunk;
  return (p.nz + kchunk - 1) / kchunk;
}

template <typename Real>
hipError_t launch_zderiv_typed(const KParams& p, const double* f, void* dz, hipStream_t s) {
  const int kchunk = 32;
  const int nchunk = (p.nz + kchunk - 1) / kchunk;
  dim3 grid(unsigned(p.splane / 256), NF, nchunk);
  hipLaunchKernelGGL(k_zderiv<Real>, grid, dim3(256), 0, s, f, static_cast<Real*>(dz), p, kchunk);
  return hipGetLastError();
}

template <typename Real, bool SOLAR>
hipError_t launch_typed(const KParams& p, int stage, const double* f, const void* dzv,
                        double* fo, double* dF, const double* uh, const double* ah, StageArgs st,
                        hipStream_t s) {
  int kchunk;
  const int nchunk = zchunks(p, 2048, kchunk);
  dim3 grid(p.nx / TX, p.ny / TY, nchunk);
  const Real* dz = static_cast<const Real*>(dzv);
  if (stage == 0)
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, false, true>), grid, dim3(NT), 0, s, f, dz, fo, dF,
                       uh, ah, p, st, kchunk);
  else if (stage == 1)
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, true, true>), grid, dim3(NT), 0, s, f, dz, fo, dF,
                       uh, ah, p, st, kchunk);
  else
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, true, false>), grid, dim3(NT), 0, s, f, dz, fo, dF,
                       uh, ah, p, st, kchunk);
  return hipGetLastError();
}

}  // namespace

size_t zderiv_bytes(const KParams& p, int prec) {
  const size_t el = prec == CMHD_FP32_SPLIT ? sizeof(float) : sizeof(double);
  return size_t(NZSLOT) * size_t(p.nz) * size_t(p.splane) * el;
}

hipError_t launch_zderiv(const KParams& p, int prec, const double* f, void* dz, hipStream_t s) {
  return prec == CMHD_FP32_SPLIT ? launch_zderiv_typed<float>(p, f, dz, s)
                                 : launch_zderiv_typed<double>(p, f, dz, s);
}

hipError_t launch_rhs_rk(const KParams& p, int prec, int stage, const double* f, const void* dz,
                         double* fo, double* dF, const double* uh, const double* ah,
                         StageArgs st, hipStream_t s) {
  if (prec == CMHD_FP32_SPLIT)
    return p.solar ? launch_typed<float, true>(p, stage, f, dz, fo, dF, uh, ah, st, s)
                   : launch_typed<float, false>(p, stage, f, dz, fo, dF, uh, ah, st, s);
  return p.solar ? launch_typed<double, true>(p, stage, f, dz, fo, dF, uh, ah, st, s)
                 : launch_typed<double, false>(p, stage, f, dz, fo, dF, uh, ah, st, s);
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
