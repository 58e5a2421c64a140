// The fused kernel of one 2N-RK3 substage (the z derivatives it reads come
// from k_zderiv, zderiv.hip).
//
// k_rhs_rk: one thread per (x, y) column of a 16 x 16 tile, marching in z.
// Every input it needs at plane k is single-plane data, staged into LDS by
// direct global->LDS copies (16-byte lanes, no registers in flight):
//   P   the 8 fields on the 22 x 24 haloed plane (x0-4 .. x0+19, y0-3 .. y0+18)
//   Zs  d/dz of A, u, ln T on the same haloed plane (for the xz, yz mixed
//       derivatives D1_x D1_z, D1_y D1_z)
//   Zo  d/dz ln rho and the 8 d2/dz2 at the own columns
// each split into the fields of A and the others (separate LDS objects, so
// that the compiler can tell a read of one from a copy in flight into the
// other).  The RK register of the own column (substages 2 and 3) is loaded
// into registers at the top of each plane and used at its end.  Per plane:
//   1a  stencils -> the pointwise inputs of all fields but A in registers;
//       D1_x of the six fields with an xy mixed derivative on the tile and its
//       y halo -> LDS
//   --  barrier; copies of the non-A fields of plane k+1 are issued (their
//       arrays were last read in 1a)
//   2a  the magnetic part of the right-hand side, A's derivatives read from
//       LDS on demand
//   --  barrier; copies of the A fields of plane k+1 are issued
//   2b  xy mixed derivatives D1_y (D1_x f) of u_x, u_y, ln T (from the D1_x
//       array, which no copy writes), radiative loss (table in LDS) and the
//       fluid part of the right-hand side from registers: the work that
//       needs no staged plane, placed where it overlaps the A copies
//   --  wait for the copies, barrier
//   3   dF <- alpha dF + dt RHS, f_next <- f + beta dF in float64, stored once
// The arithmetic of every derivative is that of the product stencils applied
// to the float64 state (differences formed in float64, then rounded to the
// precision of the right-hand side).
#include "launch.h"
#include "qslots.h"
#include "rhs_point.h"

namespace cmhd {
namespace {

// haloed plane: RW x RH, x from x0-4 (16-byte aligned rows), y from y0-3
constexpr int RW = 24, RH = 22, RPL = RW * RH;
constexpr int DXW = TX, DXH = RH;   // D1_x on the tile columns and all 22 rows
constexpr int DXP = DXW * DXH;
constexpr int NA = 3;               // fields of A
constexpr int NN = NF - NA;         // u_x u_y u_z ln rho ln T
constexpr int NZN = 4;              // haloed d/dz of u_x u_y u_z ln T
constexpr int NON = 6;              // own d/dz ln rho, d2/dz2 of u_x u_y u_z ln rho ln T
constexpr int NDX = 6;              // xy mixed: A_x A_y A_z u_x u_y ln T
constexpr int PC = NG * RW + NG;    // own point relative to a haloed-plane base
constexpr int DC = NG * DXW;        // own point relative to the D1_x base

// haloed d/dz slot of a non-A field, own-column slot of a non-A quantity
__device__ __forceinline__ constexpr int zn_index(int f) { return f == LT ? 3 : f - UX; }
__device__ __forceinline__ constexpr int on_d2(int f) { return f - UX + 1; }   // d2/dz2 of u.., ln rho, ln T
__device__ __forceinline__ constexpr int dx_index(int f) { return f <= UY ? f : (f == LT ? 5 : -1); }

// An integer the compiler cannot see through, re-made at every plane: array
// accesses are then a per-array base register plus small non-negative
// immediates, and no per-offset addresses are precomputed and held across the
// plane loop.
__device__ __forceinline__ int opaque(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

template <typename Ptr>
__device__ __forceinline__ auto d1u(Ptr a, int c, int s) {
  using R = typename std::remove_cv<typename std::remove_reference<decltype(a[0])>::type>::type;
  return R(45.0) * (a[c + s] - a[c - s]) - R(9.0) * (a[c + 2 * s] - a[c - 2 * s]) +
         (a[c + 3 * s] - a[c - 3 * s]);
}
template <typename Ptr>
__device__ __forceinline__ double d2u(Ptr a, int c, int s) {
  return -490.0 * a[c] + 270.0 * (a[c + s] + a[c - s]) - 27.0 * (a[c + 2 * s] + a[c - 2 * s]) +
         2.0 * (a[c + 3 * s] + a[c - 3 * s]);
}

// Workgroup barrier for LDS traffic only: this wave's LDS reads and writes
// are complete, global->LDS copies in flight are not waited for.  The waits
// are builtins (not asm) so that the compiler's own wait insertion knows
// about them.  s_waitcnt immediates (gfx9 encoding): lgkmcnt(0) alone is
// 0xC07F, vmcnt(0) lgkmcnt(0) is 0x0070.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wait for this wave's global->LDS copies (and stores), then a barrier: the
// copies of all waves are visible to all.
__device__ __forceinline__ void copies_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0070);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
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

// This wave's share of the copies of one plane: wave w issues the chunk
// groups m = w, w+4 of every array.  The lane offset goes through an empty asm
// so that each address stays a uniform base plus a 32-bit lane offset (no
// per-lane 64-bit pointers carried across the plane loop).
template <typename Real>
struct Copier {
  using CD = Chunks<8>;
  using CR = Chunks<sizeof(Real)>;
  unsigned hd[2], hr[2], orl;
  int w, lane;
  __device__ void init(int w_, int lane_, int x0, int y0, int nx, int ny) {
    w = w_;
    lane = lane_;
    hd[0] = CD::halo(w, lane, x0, y0, nx, ny);
    hd[1] = CD::halo(w + 4, lane, x0, y0, nx, ny);
    hr[0] = CR::halo(w, lane, x0, y0, nx, ny);
    hr[1] = CR::halo(w + 4, lane, x0, y0, nx, ny);
    orl = CR::own(w, lane, x0, y0, nx);
  }
  template <int E>
  __device__ void halo(const void* base, void* lds, unsigned off0, unsigned off1) const {
    using C = Chunks<E>;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int m = w + 4 * g;
      unsigned off = g == 0 ? off0 : off1;
      asm volatile("" : "+v"(off));
      if (m < C::HI && m * 64 + lane < C::HN)
        copy16(static_cast<const char*>(base) + off, static_cast<char*>(lds) + m * 1024);
    }
  }
  template <int E>
  __device__ void own(const void* base, void* lds, unsigned off) const {
    using C = Chunks<E>;
    asm volatile("" : "+v"(off));
    if (w < C::OI && w * 64 + lane < C::ON)
      copy16(static_cast<const char*>(base) + off, static_cast<char*>(lds) + w * 1024);
  }
};

// The radiative-loss table copied into LDS.
struct LdsRadTable {
  const double* t;   // [lnT 16][lnL 16][slope 16]
  __device__ __forceinline__ double lnT(int i) const { return t[i]; }
  __device__ __forceinline__ double lnL(int i) const { return t[CMHD_MAX_RAD + i]; }
  __device__ __forceinline__ double slope(int i) const { return t[2 * CMHD_MAX_RAD + i]; }
};

// The initial profiles of the Newtonian cooling copied into LDS.
struct LdsNcTable {
  const double* t;   // [ln rho0 (n)][ln T0 (n)]
  int n;
  __device__ __forceinline__ double lnrho0(int i) const { return t[i]; }
  __device__ __forceinline__ double lnT0(int i) const { return t[n + i]; }
};

// Source for rhs_eval: the derivatives of A are read from the staged plane on
// demand (rolled component loop, few registers), everything else from the
// inputs gathered into registers (indices are compile-time constants).  The
// A arrays are addressed from per-plane opaque bases at their lowest address.
template <typename Real>
struct HybridSource {
  static constexpr int kUnrollA = 1, kUnrollU = 3;
  const Real* q;
  const double* v64s;
  const double* pP;   // A fields, haloed plane, based at c - PC
  const Real* pZ;     // d/dz of A, haloed, based at c - PC
  const Real* pO;     // d2/dz2 of A, own column
  const double* pD;   // D1_x, based at cx - DC
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
        case 0: return Real(d2u(pP, b, 1) * i180dx2);
        case 1: return Real(d2u(pP, b, RW) * i180dy2);
        case 2: return pO[f * NT];
        case 3: return Real(d1u(pD, f * DXP + DC, DXW) * ixy);
        case 4: return d1u(pZ, b, 1) * Real(i60dx);
        default: return d1u(pZ, b, RW) * Real(i60dy);
      }
    }
    const int slot = q_h(f, s);
    return slot >= 0 ? q[slot] : Real(0.0);
  }
  __device__ __forceinline__ Real lapr() const { return q[Q_LAPR]; }
};

// Block -> (tile x, tile y, z chunk).  Blocks are dispatched round-robin to
// the 8 XCDs (each with its own L2), and the 32 CUs of an XCD run 32 blocks at
// a time.  With the XCD-aware order, the blocks that one XCD runs together form
// a compact patch of pw x ph tiles of one z chunk, so that the haloed rows they
// share (three 128-byte lines per 24-element row) are L2 hits and not
// separate HBM reads.
struct TileMap {
  int ntx, nty, pw, ph, xcd;
};

__device__ __forceinline__ void tile_of(int id, const TileMap& m, int& bx, int& by, int& bz) {
  if (m.xcd) {
    const int np = m.pw * m.ph;
    const int slot = id >> 3;
    const int patch = (slot / np) * 8 + (id & 7);
    const int within = slot - (slot / np) * np;
    const int ppr = m.ntx / m.pw;
    const int ppc = ppr * (m.nty / m.ph);
    bz = patch / ppc;
    const int r = patch - bz * ppc;
    bx = (r % ppr) * m.pw + within % m.pw;
    by = (r / ppr) * m.ph + within / m.pw;
  } else {
    bx = id % m.ntx;
    by = (id / m.ntx) % m.nty;
    bz = id / (m.ntx * m.nty);
  }
}

__device__ __forceinline__ void swamp(const KParams& p, int k, double& w, double& dw) {
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

// ---------------------------------------------------------------------------
template <typename Real, bool SOLAR, bool READ_DF, bool WRITE_DF, bool NEWTON>
__global__ __launch_bounds__(NT) void k_rhs_rk(const double* __restrict__ f,
                                               const Real* __restrict__ dz,
                                               double* __restrict__ fo,
                                               double* __restrict__ dF,
                                               const double* __restrict__ uh,
                                               const double* __restrict__ ah, const KParams p,
                                               const StageArgs st, int kchunk, int chunk0,
                                               const TileMap tm) {
  __shared__ __align__(16) double sPA[NA][RPL];   // values of A, haloed
  __shared__ __align__(16) double sPN[NN][RPL];   // values of u, ln rho, ln T, haloed
  __shared__ __align__(16) Real sZA[NA][RPL];     // d/dz of A, haloed
  __shared__ __align__(16) Real sZN[NZN][RPL];    // d/dz of u, ln T, haloed
  __shared__ __align__(16) Real sOA[NA][NT];      // d2/dz2 of A, own
  __shared__ __align__(16) Real sON[NON][NT];     // d/dz ln rho, d2/dz2 of the others, own
  __shared__ __align__(16) double sDx[NDX][DXP];  // D1_x (unscaled) on tile + y halo
  __shared__ __align__(16) double sRad[3 * CMHD_MAX_RAD];
  // Newtonian cooling profiles (only the NEWTON variant has the term)
  __shared__ __align__(16) double sNC[NEWTON ? 2 * CMHD_MAX_NC_TABLE : 1];

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  int bx, by, bz;
  tile_of(blockIdx.x, tm, bx, by, bz);
  const int x0 = bx * TX, y0 = by * TY;
  const long long sp = p.splane, sf = p.sfield, szs = (long long)p.nz * sp;
  const int oc = (y0 + ty) * p.nx + (x0 + tx);    // own column within a plane
  const int c = (ty + NG) * RW + (tx + 4);        // own point in the haloed plane
  const int cx = (ty + NG) * DXW + tx;            // own point in the D1_x array

  Copier<Real> cp;
  cp.init(__builtin_amdgcn_readfirstlane(tid / 64), tid % 64, x0, y0, p.nx, p.ny);
  // copies of plane k: the fields of A (a) or the others
  auto copy_plane = [&](int k, bool a) {
    if (a) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        cp.template halo<8>(f + (AX + i) * sf + (k + NG) * sp, sPA[i], cp.hd[0], cp.hd[1]);
        cp.template halo<sizeof(Real)>(dz + (AX + i) * szs + k * sp, sZA[i], cp.hr[0], cp.hr[1]);
        cp.template own<sizeof(Real)>(dz + (NF + AX + i) * szs + k * sp, sOA[i], cp.orl);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NN; ++i)
        cp.template halo<8>(f + (UX + i) * sf + (k + NG) * sp, sPN[i], cp.hd[0], cp.hd[1]);
#pragma unroll
      for (int i = 0; i < NZN; ++i) {
        const int fi = i < 3 ? UX + i : LT;
        cp.template halo<sizeof(Real)>(dz + fi * szs + k * sp, sZN[i], cp.hr[0], cp.hr[1]);
      }
      cp.template own<sizeof(Real)>(dz + LR * szs + k * sp, sON[0], cp.orl);
#pragma unroll
      for (int i = 0; i < NN; ++i)
        cp.template own<sizeof(Real)>(dz + (NF + UX + i) * szs + k * sp, sON[1 + i], cp.orl);
    }
  };

  // y-halo rows of D1_x computed by threads 0..95: rows 0-2 and 19-21
  const int hrow = tid < 3 * TX ? tid / TX : TY + NG + (tid - 3 * TX) / TX;
  const int hcol = tid % TX;

  const int kbeg = (chunk0 + bz) * kchunk;
  const int kend = min(kbeg + kchunk, p.nz);

  if (tid < CMHD_MAX_RAD) {
    sRad[tid] = p.rad_lnT[tid];
    sRad[CMHD_MAX_RAD + tid] = p.rad_lnL[tid];
    sRad[2 * CMHD_MAX_RAD + tid] = p.rad_slope[tid];
  }
  if (NEWTON)
    for (int i = tid; i < 2 * p.nc_n; i += NT) sNC[i] = p.nc_tab[i];
  copy_plane(kbeg, true);
  copy_plane(kbeg, false);
  copies_barrier();

  for (int k = kbeg; k < kend; ++k) {
    // the RK register of the own column, loaded at the top of the plane and
    // consumed by the update at its end (registers, no LDS staging)
    double dfr[NF];
    if (READ_DF) {
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) dfr[fi] = dF[fi * sf + (k + NG) * sp + oc];
    }
    // ---- 1a: stencils of the staged plane into registers (all but the
    // derivatives of A); D1_x of the xy-mixed fields into LDS
    const int ic = opaque(c - PC), icx = opaque(cx - DC), it = opaque(tid);
    const double* pPA = &sPA[0][0] + ic;
    const double* pPN = &sPN[0][0] + ic;
    const Real* pZN = &sZN[0][0] + ic;
    const Real* pON = &sON[0][0] + it;
    double* pDx = &sDx[0][0] + icx;
    Real q[NQ];
    double v64[NF];
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const double* pP = fi <= AZ ? pPA : pPN;
      const int b = (fi <= AZ ? fi : fi - UX) * RPL + PC;
      const double c0 = pP[b];
      const double d1x = d1u(pP, b, 1);
      v64[fi] = c0;
      q[q_v(fi)] = Real(c0);
      q[q_d(fi, 0)] = Real(d1x * p.i60dx);
      if (dx_index(fi) >= 0) pDx[dx_index(fi) * DXP + DC] = d1x;
      if (fi > AZ) {
        q[q_d(fi, 1)] = Real(d1u(pP, b, RW) * p.i60dy);
        const double d2x = d2u(pP, b, 1), d2y = d2u(pP, b, RW);
        if (fi == LR) {
          q[q_d(fi, 2)] = pON[0];
          q[Q_LAPR] = Real(d2x * p.i180dx2 + d2y * p.i180dy2 + double(pON[on_d2(LR) * NT]));
        } else {
          const int zb = zn_index(fi) * RPL + PC;
          q[q_d(fi, 2)] = pZN[zb];
          q[q_h(fi, 0)] = Real(d2x * p.i180dx2);
          q[q_h(fi, 1)] = Real(d2y * p.i180dy2);
          q[q_h(fi, 2)] = pON[on_d2(fi) * NT];
          if (q_h(fi, 4) >= 0) q[q_h(fi, 4)] = d1u(pZN, zb, 1) * Real(p.i60dx);
          if (q_h(fi, 5) >= 0) q[q_h(fi, 5)] = d1u(pZN, zb, RW) * Real(p.i60dy);
        }
      }
    }
    // D1_x on the y-halo rows (threads 0..95)
    if (tid < 2 * NG * TX) {
      const int ih = opaque(hrow * RW + hcol + 4 - NG), ihx = opaque(hrow * DXW + hcol);
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        if (dx_index(fi) < 0) continue;
        const double* pP = (fi <= AZ ? &sPA[0][0] : &sPN[0][0]) + ih;
        const int b = (fi <= AZ ? fi : fi - UX) * RPL + NG;
        (&sDx[0][0] + ihx)[dx_index(fi) * DXP] = d1u(pP, b, 1);
      }
    }
    lds_barrier();

    // ---- copies into the arrays last read in 1a: the non-A fields of the
    // next plane
    if (k + 1 < kend) copy_plane(k + 1, false);

    const double ixy = p.i60dx * p.i60dy;

    // ---- 2a: the magnetic part (A read from LDS)
    PointCtx<Real> pc;
    swamp(p, k, pc.w, pc.dw);
    pc.bottom = SOLAR && k == 0;
    pc.top = SOLAR && k == p.nz - 1;
    pc.ramp = st.ramp;
    pc.nc_cz = NEWTON ? nc_height_cut(p, k) : 0.0;
    pc.nc_lnT0 = NEWTON ? sNC[p.nc_n + k + NG] : 0.0;
    if (SOLAR && k == 0) {
      pc.uh[0] = Real(uh[oc]);
      pc.uh[1] = Real(uh[sp + oc]);
      pc.ah[0] = Real(ah[oc]);
      pc.ah[1] = Real(ah[sp + oc]);
    } else {
      pc.uh[0] = pc.uh[1] = pc.ah[0] = pc.ah[1] = Real(0.0);
    }
    const HybridSource<Real> src{q, v64, pPA, &sZA[0][0] + ic, &sOA[0][0] + it, pDx,
                                 p.i60dx, p.i60dy, p.i180dx2, p.i180dy2, ixy};
    Real out[NF];
    MagState<Real> mag;
    rhs_magnetic<Real>(src, pc, p, out, mag);
    lds_barrier();

    // ---- copies of the A fields of the next plane
    if (k + 1 < kend) copy_plane(k + 1, true);

    // ---- 2b: xy mixed derivatives D1_y (D1_x f) of u_x, u_y, ln T, radiative
    // loss and the fluid part of the right-hand side, while the copies land
#pragma unroll
    for (int fi = UX; fi < NF; ++fi)
      if (dx_index(fi) >= 0) q[q_h(fi, 3)] = Real(d1u(pDx, dx_index(fi) * DXP + DC, DXW) * ixy);
    const Real rad = rhs_radiation<Real>(src, p, LdsRadTable{sRad});
    const Real nc = NEWTON ? rhs_newton<Real>(src, p, LdsNcTable{sNC, p.nc_n}, pc) : Real(0.0);
    rhs_fluid<Real>(src, pc, p, mag, rad, nc, out);

    copies_barrier();

    // ---- 3: 2N-RK3 register update in float64
    const unsigned ob = unsigned(oc) * 8u;   // byte offset of the own column
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const long long pl = fi * sf + (k + NG) * sp;   // uniform
      const double r = double(out[fi]);
      double d = READ_DF ? st.alpha * dfr[fi] + st.dt * r : st.dt * r;
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

template <typename Real, bool SOLAR, bool NEWTON>
hipError_t launch_typed(const KParams& p, int stage, const double* f, const void* dzv,
                        double* fo, double* dF, const double* uh, const double* ah, StageArgs st,
                        const ChunkPlan& cp, int chunk0, int nchunks, hipStream_t s) {
  TileMap tm{p.nx / TX, p.ny / TY, 8, 4, 0};
  tm.pw = tm.ntx < tm.pw ? tm.ntx : tm.pw;
  tm.ph = tm.nty < tm.ph ? tm.nty : tm.ph;
  // XCD-aware order when the patches split evenly over the 8 XCDs
  tm.xcd = ((tm.ntx / tm.pw) * (tm.nty / tm.ph) * nchunks) % 8 == 0;
  dim3 grid(unsigned(tm.ntx * tm.nty * nchunks));
  const Real* dz = static_cast<const Real*>(dzv);
  if (stage == 0)
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, false, true, NEWTON>), grid, dim3(NT), 0, s, f, dz,
                       fo, dF, uh, ah, p, st, cp.kchunk, chunk0, tm);
  else if (stage == 1)
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, true, true, NEWTON>), grid, dim3(NT), 0, s, f, dz,
                       fo, dF, uh, ah, p, st, cp.kchunk, chunk0, tm);
  else
    hipLaunchKernelGGL((k_rhs_rk<Real, SOLAR, true, false, NEWTON>), grid, dim3(NT), 0, s, f, dz,
                       fo, dF, uh, ah, p, st, cp.kchunk, chunk0, tm);
  return hipGetLastError();
}

// the Newtonian cooling variant is built for the solar (stratified) mode only
template <typename Real>
hipError_t launch_prec(const KParams& p, int stage, const double* f, const void* dz, double* fo,
                       double* dF, const double* uh, const double* ah, StageArgs st,
                       const ChunkPlan& cp, int chunk0, int nchunks, hipStream_t s) {
  if (p.solar && p.nc_tau != 0.0)
    return launch_typed<Real, true, true>(p, stage, f, dz, fo, dF, uh, ah, st, cp, chunk0, nchunks, s);
  if (p.solar)
    return launch_typed<Real, true, false>(p, stage, f, dz, fo, dF, uh, ah, st, cp, chunk0, nchunks, s);
  return launch_typed<Real, false, false>(p, stage, f, dz, fo, dF, uh, ah, st, cp, chunk0, nchunks, s);
}

}  // namespace

ChunkPlan plan_chunks(const KParams& p) {
  ChunkPlan c;
  const int tiles = (p.nx / TX) * (p.ny / TY);
  if (tiles >= 256 && p.nz >= 32) {
    // pipelined: z chunks of an eighth of the box (at least 16 planes), one
    // fused launch per chunk of all tiles (8 chunks measured faster than 2, 4
    // or 16 at 512^2 x 256)
    c.kchunk = (p.nz + 7) / 8;
    c.kchunk = c.kchunk < 16 ? 16 : c.kchunk;
    c.nchunk = (p.nz + c.kchunk - 1) / c.kchunk;
    c.pipelined = true;
  } else {
    // one launch of about 2048 blocks
    int nchunk = (2048 + tiles - 1) / tiles;
    if (nchunk > p.nz) nchunk = p.nz;
    c.kchunk = (p.nz + nchunk - 1) / nchunk;
    c.nchunk = (p.nz + c.kchunk - 1) / c.kchunk;
    c.pipelined = false;
  }
  return c;
}

hipError_t launch_rhs_rk(const KParams& p, int prec, int stage, const double* f, const void* dz,
                         double* fo, double* dF, const double* uh, const double* ah,
                         StageArgs st, const ChunkPlan& cp, int chunk0, int nchunks,
                         hipStream_t s) {
  if (prec == CMHD_FP32_SPLIT)
    return launch_prec<float>(p, stage, f, dz, fo, dF, uh, ah, st, cp, chunk0, nchunks, s);
  return launch_prec<double>(p, stage, f, dz, fo, dF, uh, ah, st, cp, chunk0, nchunks, s);
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
