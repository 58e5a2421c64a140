// One 2N-RK3 substage in one kernel: stencils, pointwise right-hand side and
// register update, with the z derivatives formed on chip from a sliding
// window of each column (no z-derivative buffer in HBM).
//
// k_substage: one block of 1024 threads (16 waves, four per SIMD) per 16 x 16
// tile of columns and z chunk, marching in z.  Waves 8-15 hold the z window,
// waves 0-3 evaluate the magnetic part of the right-hand side, waves 4-7 the
// fluid part.  Per plane k:
//
//   W  window: thread t < 484 owns column t of the 22 x 22 haloed tile and
//      keeps the planes k-3 .. k+3 of all 8 fields in registers (each
//      loaded once, from HBM/L2, during the previous plane).  It writes to
//      LDS the plane values f(k), the sixth-order d/dz on the haloed tile
//      and, for the own columns, d2/dz2 (metric-scaled on a non-uniform
//      grid).
//      Meanwhile the right-hand-side waves finish plane k-1 (F below).
//   X  D1_x of the six fields with an xy mixed derivative (A, u_x, u_y,
//      ln T) on the tile columns and all 22 rows, those of A_x, A_y by the
//      window waves, which then load the next plane into their ring, the others
//      by the right-hand-side waves, which also copy the RK register and f
//      of the own tile into LDS and form the pointwise terms: the radiative
//      loss and 1/rho (magnetic waves), the parts of continuity and energy
//      without div u and S:S, the Newtonian cooling, T and 1/(c_v T)
//      (fluid).
//   R  right-hand side at the own columns, every derivative read from LDS
//      on demand: the magnetic waves the induction equation, B, J, Spitzer
//      conduction, Ohmic heating, the swamp diffusion of ln T and the Lorentz
//      force; the fluid waves the momentum equation and the div u and S:S
//      terms.  Results go to LDS.
//   F  (during the next plane's W) from LDS only: the fluid waves add the
//      magnetic terms and the boundary terms; both update their fields.
//
// Three barriers per plane (after W, after X, after R).  The HBM traffic is
// that of the 2N method itself: f read once (halo columns of neighbouring
// tiles are shared through L2; the own-column copy for F is an L2 hit), dF
// read and written, f_next written, 213 B per zone and substage on average.
//
// Mixed derivatives are products of first-derivative stencils: xy as D1_y of
// the staged D1_x, xz and yz as D1_x, D1_y of the staged d/dz.  Every
// stencil sum is formed in float64 from the float64 state and rounded to the
// precision of the right-hand side (float in the split form) afterwards.
#include "launch.h"
#include "qslots.h"
#include "rhs_point.h"

namespace cmhd {
namespace {

constexpr int HW = TX + 2 * NG;      // 22: haloed tile width and height
constexpr int HN = HW * HW;          // 484 haloed columns
constexpr int NT2 = 2 * NT;          // 512: threads of the RHS waves, and of the window waves
constexpr int NTB = 4 * NT;          // 1024 threads per block
constexpr int OWN = NG * HW + NG;    // haloed index of the tile's first own column
constexpr int NDX = 6;               // fields with an xy mixed derivative
constexpr int DXP = TX * HW;         // D1_x on the tile columns and all 22 rows
constexpr int DOWN = NG * TX;        // D1_x index of the tile's first own column
constexpr int NXCH = 4;              // values per zone from the magnetic to the fluid waves

__host__ __device__ constexpr int dx_slot(int f) {
  return f <= UY ? f : (f == LT ? 5 : -1);
}
__host__ __device__ constexpr int dx_field(int s) { return s < 5 ? s : LT; }


template <typename Real, bool NEWTON>
struct Smem {
  double P[NF][HN];         // f(k) on the haloed tile
  Real Z[NF][HN];           // d/dz on the haloed tile (ln rho: own columns only)
  Real ZZ[NF][NT];          // d2/dz2 at the own columns
  double Dx[NDX][DXP];      // unscaled D1_x
  Real X[NXCH][NT];         // magnetic -> fluid
  Real Q[9][NT];            // momentum RHS (3), d ln rho/dt, d ln T/dt (partial), radiative loss,
                            // T, 1/(c_v T), 1/rho
  Real QA[3][NT];           // induction RHS
  double R[NF][NT];         // the RK register of the own columns (global->LDS copies)
  double Fown[NF][NT];      // f at the own columns (global->LDS copies)
  double rad[3 * CMHD_MAX_RAD];
};

// An integer the compiler cannot see through, re-made at every plane, so that
// array accesses are a per-array base register plus small non-negative
// immediates and no per-offset addresses are held across the plane loop.
__device__ __forceinline__ int opaque(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

// A wave-uniform double the compiler re-reads from its scalar register at
// each use (its conversion to float is then not hoisted into a vector
// register held across the plane loop)
__device__ __forceinline__ double sreg(double x) {
  asm volatile("" : "+s"(x));
  return x;
}

// Workgroup barrier for LDS traffic only: this wave's LDS reads and writes
// are complete; global loads in flight (the next plane's window) are not
// waited for.  s_waitcnt lgkmcnt(0) alone is 0xC07F in the gfx9 encoding.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wait for this wave's global->LDS copies (and all its other vector memory
// operations), then a barrier: the copies of all waves are visible to all.
// The compiler inserts no wait of its own for such a copy before an LDS read
// of its destination; this is the only guard.  vmcnt(0) lgkmcnt(0) is 0x0070.
__device__ __forceinline__ void copies_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0x0070);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// one 16-byte global->LDS copy per lane: lane l writes lds_base + 16 l (the
// destination is wave-uniform); gsrc is the lane's own source address
__device__ __forceinline__ void copy16(const void* gsrc, void* lds_base) {
  __builtin_amdgcn_global_load_lds(gsrc, (__attribute__((address_space(3))) void*)lds_base, 16,
                                   0, 0);
}

// unscaled sixth-order first and second differences along stride s around a[0]
template <typename T>
__device__ __forceinline__ T d1s(const T* a, int s) {
  return T(45.0) * (a[s] - a[-s]) - T(9.0) * (a[2 * s] - a[-2 * s]) + (a[3 * s] - a[-3 * s]);
}

// the same first difference with at most two of its values in flight (the
// window waves form it while they hold their z window in registers)
template <typename T>
__device__ __forceinline__ T d1s_lean(const T* a, int s) {
  T acc = T(45.0) * (a[s] - a[-s]);
  __builtin_amdgcn_sched_barrier(0);
  acc = acc - T(9.0) * (a[2 * s] - a[-2 * s]);
  __builtin_amdgcn_sched_barrier(0);
  return acc + (a[3 * s] - a[-3 * s]);
}

// Global access at a wave-uniform base plus a 32-bit per-lane byte offset
// (scalar base register + one offset register, no per-lane 64-bit pointers)
// (the empty asm keeps the compiler from folding the offset into a 64-bit
// per-lane pointer)
template <typename T>
__device__ __forceinline__ T ld_u(const T* ubase, unsigned off) {
  asm volatile("" : "+v"(off));
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(ubase) + off);
}
template <typename T>
__device__ __forceinline__ void st_u(T* ubase, unsigned off, T v) {
  asm volatile("" : "+v"(off));
  *reinterpret_cast<T*>(reinterpret_cast<char*>(ubase) + off) = v;
}

// the radiative-loss table and the Newtonian-cooling profiles copied into LDS
struct LdsRadTable {
  const double* t;   // [lnT 16][lnL 16][slope 16]
  __device__ __forceinline__ double lnT(int i) const { return t[i]; }
  __device__ __forceinline__ double lnL(int i) const { return t[CMHD_MAX_RAD + i]; }
  __device__ __forceinline__ double slope(int i) const { return t[2 * CMHD_MAX_RAD + i]; }
};

// Source of the pointwise right-hand side: every value and derivative read
// from LDS on demand.  Bases are per-thread (tile origin of the own column)
// so that all stencil offsets are non-negative immediates.
template <typename Real>
struct LdsSrc {
  static constexpr int kUnrollA = 1, kUnrollU = 1;
  const double* P;    // + f*HN + OWN: own column
  const Real* Z;      // + f*HN + OWN
  const Real* ZZ;     // + f*NT
  const double* Dx;   // + s*DXP + DOWN
  double i60dx, i60dy, i180dx2, i180dy2, ixy;

  __device__ __forceinline__ Real v(int f) const { return Real(P[f * HN + OWN]); }
  __device__ __forceinline__ double v64(int f) const { return P[f * HN + OWN]; }
  __device__ __forceinline__ Real d(int f, int dir) const {
    const double* a = P + f * HN + OWN;
    if (dir == 0) return Real(d1s(a, 1) * i60dx);
    if (dir == 1) return Real(d1s(a, HW) * i60dy);
    return Z[f * HN + OWN];
  }
  // the gradient of f, its reads issued together and waited for once
  __device__ __forceinline__ void grad(int f, Real g[3]) const {
    const double* a = P + f * HN + OWN;
    const double p1 = a[1], m1 = a[-1], p2 = a[2], m2 = a[-2], p3 = a[3], m3 = a[-3];
    const double q1 = a[HW], n1 = a[-HW], q2 = a[2 * HW], n2 = a[-2 * HW], q3 = a[3 * HW],
                 n3 = a[-3 * HW];
    const Real zc = Z[f * HN + OWN];
    __builtin_amdgcn_sched_barrier(0);
    g[0] = Real((45.0 * (p1 - m1) - 9.0 * (p2 - m2) + (p3 - m3)) * i60dx);
    g[1] = Real((45.0 * (q1 - n1) - 9.0 * (q2 - n2) + (q3 - n3)) * i60dy);
    g[2] = zc;
  }
  __device__ __forceinline__ static double d2x(const double* a) {
    return -490.0 * a[0] + 270.0 * (a[1] + a[-1]) - 27.0 * (a[2] + a[-2]) +
           2.0 * (a[3] + a[-3]);
  }
  __device__ __forceinline__ static double d2y(const double* a) {
    return -490.0 * a[0] + 270.0 * (a[HW] + a[-HW]) - 27.0 * (a[2 * HW] + a[-2 * HW]) +
           2.0 * (a[3 * HW] + a[-3 * HW]);
  }
  // gradient and Hessian of f; the seven x (y) values serve both D1 and D2.
  // The reads are issued in two batches (the plane values and the z
  // derivatives, then the mixed-derivative stencils), each waited for once.
  __device__ __forceinline__ void gh(int f, Real g[3], Real hh[6]) const {
    const double* a = P + f * HN + OWN;
    const double c = a[0], p1 = a[1], m1 = a[-1], p2 = a[2], m2 = a[-2], p3 = a[3], m3 = a[-3];
    const double q1 = a[HW], n1 = a[-HW], q2 = a[2 * HW], n2 = a[-2 * HW], q3 = a[3 * HW],
                 n3 = a[-3 * HW];
    const Real zc = Z[f * HN + OWN], zzc = ZZ[f * NT];
    __builtin_amdgcn_sched_barrier(0);
    g[0] = Real((45.0 * (p1 - m1) - 9.0 * (p2 - m2) + (p3 - m3)) * i60dx);
    hh[0] = Real((-490.0 * c + 270.0 * (p1 + m1) - 27.0 * (p2 + m2) + 2.0 * (p3 + m3)) *
                 i180dx2);
    g[1] = Real((45.0 * (q1 - n1) - 9.0 * (q2 - n2) + (q3 - n3)) * i60dy);
    hh[1] = Real((-490.0 * c + 270.0 * (q1 + n1) - 27.0 * (q2 + n2) + 2.0 * (q3 + n3)) *
                 i180dy2);
    g[2] = zc;
    hh[2] = zzc;
    __builtin_amdgcn_sched_barrier(0);
    hh[3] = q_h(f, 3) >= 0 && dx_slot(f) >= 0
                ? Real(d1s(Dx + dx_slot(f) * DXP + DOWN, TX) * ixy)
                : Real(0);
    hh[4] = q_h(f, 4) >= 0 ? d1s(Z + f * HN + OWN, 1) * Real(i60dx) : Real(0);
    hh[5] = q_h(f, 5) >= 0 ? d1s(Z + f * HN + OWN, HW) * Real(i60dy) : Real(0);
  }
  __device__ __forceinline__ Real lapr() const {
    const double* a = P + LR * HN + OWN;
    return Real(d2x(a) * i180dx2 + d2y(a) * i180dy2 + double(ZZ[LR * NT]));
  }
};

// f at the own column, from the LDS copy (the boundary terms of F)
template <typename Real>
struct OwnSrc {
  const double* F;    // + f*NT: own column
  __device__ __forceinline__ Real v(int f) const { return Real(F[f * NT]); }
  __device__ __forceinline__ double v64(int f) const { return F[f * NT]; }
};

// Block -> (tile x, tile y, z chunk).  Blocks are dispatched round-robin to
// the 8 XCDs (each with its own L2), and the 32 CUs of an XCD run 32 blocks at
// a time.  With the XCD-aware order, the blocks that one XCD runs together form
// a compact patch of pw x ph tiles of one z chunk, so that the haloed rows they
// share are L2 hits and not separate HBM reads.
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

// z metric of plane k: d/dz = c1 S1, d2/dz2 = c2 S2 + c3 S1 with S1, S2 the
// unscaled stencil sums (uniform grid: 1/(60 dz), 1/(180 dz^2), 0).  The
// non-uniform table is read through the constant address space (scalar loads).
__device__ __forceinline__ void zmetric(const KParams& p, int k, double& c1, double& c2,
                                        double& c3) {
  if (!p.stretched) {
    c1 = p.i60dz;
    c2 = p.i180dz2;
    c3 = 0.0;
    return;
  }
  const __attribute__((address_space(4))) double* t =
      (const __attribute__((address_space(4))) double*)p.ztab;
  c1 = t[zt_c1(p) + k];
  c2 = t[zt_c2(p) + k];
  c3 = t[zt_c3(p) + k];
}

// D1_x (unscaled) of the xy-mixed fields on the tile columns and all 22 rows
// of the staged plane (the right-hand side reads it for the xy mixed
// derivatives), between the first and second barrier: the window waves form
// the slots [0, NDXW) with at most two values in flight (they hold their z
// window meanwhile), the right-hand-side waves the rest.  t is the thread's
// index within its group of 512.
constexpr int NDXW = 2;   // slots of the window waves
template <typename Real, bool NEWTON, bool WINDOW>
__device__ __forceinline__ void stencils_dx(Smem<Real, NEWTON>& sm, int t) {
  constexpr int s0 = WINDOW ? 0 : NDXW;
  constexpr int n = (WINDOW ? NDXW : NDX - NDXW) * DXP;
  // (opaque: the per-item indices are re-derived at every plane, not held
  // in registers across the plane loop)
#pragma unroll 1
  for (int i = opaque(t); i < n; i += NT2) {
    const int s = i / DXP + s0, pt = i - (i / DXP) * DXP;
    const int row = pt / TX, col = pt - row * TX;
    const double* a = &sm.P[dx_field(s)][row * HW + col + NG];
    sm.Dx[s][pt] = WINDOW ? d1s_lean(a, 1) : d1s(a, 1);
  }
}

// ---------------------------------------------------------------------------
// The window waves (8..15): W and X of every plane.  Each thread keeps the
// planes k-3 .. k+3 of its column in a ring of registers; the loop is unrolled
// by the ring length so that the slot of each plane is a compile-time index
// and no value moves.
template <typename Real, bool NEWTON>
__device__ __forceinline__ void window_loop(Smem<Real, NEWTON>& sm, const double* __restrict__ f,
                                            const KParams& p, int wt, int x0, int y0, int kbeg,
                                            int kend) {
  const long long sp = p.splane, sf = p.sfield;
  // window column (threads 484..511 of the window waves hold a copy of a
  // valid column and write nothing)
  const bool win = wt < HN;
  const int hx = wt % HW, hy = wt / HW;
  int gx = x0 - NG + hx, gy = y0 - NG + hy;
  gx += gx < 0 ? p.nx : 0;
  gx -= gx >= p.nx ? p.nx : 0;
  gy += gy < 0 ? p.ny : 0;
  gy -= gy >= p.ny ? p.ny : 0;
  const unsigned wc = unsigned(gy * p.nx + gx) * 8u;   // window column, bytes
  const bool wown = win && hx >= NG && hx < NG + TX && hy >= NG && hy < NG + TY;
  const int wo = (hy - NG) * TX + (hx - NG);

  // ring: at plane k, slot (r + j) % 7 holds f at interior plane k-3+j
  // (stored plane k+j), r = (k - kbeg) % 7
  double w[NF][7];
#pragma unroll
  for (int fi = 0; fi < NF; ++fi)
#pragma unroll
    for (int j = 0; j < 7; ++j) w[fi][j] = ld_u(f + fi * sf + (kbeg + j) * sp, wc);

  auto plane = [&](auto rc, int k) {
    constexpr int r = decltype(rc)::value;
    // W is the critical path of the plane; the update of the previous plane
    // shares the SIMDs with it and has slack, so the window issues first
    // until the plane is staged (the arbiter otherwise favours the older
    // right-hand-side waves)
    __builtin_amdgcn_s_setprio(2);
    double c1, c2, c3;
    zmetric(p, k, c1, c2, c3);
    // the metric's scalar loads waited for here, once: a wait inside the
    // exec-masked stores below would also drain the LDS stores before it
    c1 = sreg(c1);
    c2 = sreg(c2);
    c3 = sreg(c3);
#pragma unroll
    for (int fi = 0; fi < NF; ++fi) {
      const double q0 = w[fi][r % 7], q1 = w[fi][(r + 1) % 7], q2 = w[fi][(r + 2) % 7];
      const double q3 = w[fi][(r + 3) % 7], q4 = w[fi][(r + 4) % 7];
      const double q5 = w[fi][(r + 5) % 7], q6 = w[fi][(r + 6) % 7];
      const double s1 = 45.0 * (q4 - q2) - 9.0 * (q5 - q1) + (q6 - q0);
      const double s2 = -490.0 * q3 + 270.0 * (q4 + q2) - 27.0 * (q5 + q1) + 2.0 * (q6 + q0);
      if (win) {
        sm.P[fi][wt] = q3;
        sm.Z[fi][wt] = Real(s1 * c1);
      }
      if (wown) sm.ZZ[fi][wo] = Real(s2 * c2 + s1 * c3);
    }
    lds_barrier();   // B1: the plane is staged
    __builtin_amdgcn_s_setprio(0);
    // the stencils while the slot of plane k-3 is free, then the next
    // plane's values into it (consumed at the next plane; the last plane
    // reloads a plane it already holds: the load is unconditional)
    stencils_dx<Real, NEWTON, true>(sm, wt);
    {
      const double* fn = f + (k + 1 < kend ? k + 7 : k + 6) * sp;
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) w[fi][r] = ld_u(fn + fi * sf, wc);
    }
    lds_barrier();   // B2: the stencils are staged; the RHS waves work on the plane
    lds_barrier();   // B3: right-hand sides done, the staged plane is no longer read
  };
  for (int k = kbeg; k < kend; k += 7) {
    plane(std::integral_constant<int, 0>{}, k);
    if (k + 1 >= kend) break;
    plane(std::integral_constant<int, 1>{}, k + 1);
    if (k + 2 >= kend) break;
    plane(std::integral_constant<int, 2>{}, k + 2);
    if (k + 3 >= kend) break;
    plane(std::integral_constant<int, 3>{}, k + 3);
    if (k + 4 >= kend) break;
    plane(std::integral_constant<int, 4>{}, k + 4);
    if (k + 5 >= kend) break;
    plane(std::integral_constant<int, 5>{}, k + 5);
    if (k + 6 >= kend) break;
    plane(std::integral_constant<int, 6>{}, k + 6);
  }
}

template <typename Real, bool SOLAR, bool READ_DF, bool WRITE_DF, bool NEWTON>
__global__ __launch_bounds__(NTB) void k_substage(const double* __restrict__ f,
                                                  double* __restrict__ fo,
                                                  double* __restrict__ dF,
                                                  const double* __restrict__ uh,
                                                  const double* __restrict__ ah, const KParams p,
                                                  const StageArgs st, int kchunk,
                                                  const TileMap tm) {
  __shared__ __align__(16) Smem<Real, NEWTON> sm;

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid) / 64;   // uniform
  int bx, by, bz;
  tile_of(blockIdx.x, tm, bx, by, bz);
  const int x0 = bx * TX, y0 = by * TY;
  const int kbeg = bz * kchunk;
  const int kend = min(kbeg + kchunk, p.nz);

  if (wave >= 8) {
    window_loop<Real, NEWTON>(sm, f, p, tid - NT2, x0, y0, kbeg, kend);
    return;
  }

  // ---- the right-hand-side waves: 0-3 magnetic, 4-7 fluid
  const bool mag = wave < 4;
  const int o = mag ? tid : tid - NT;           // own column of the tile
  const int tx = o % TX, ty = o / TX;
  const long long sp = p.splane, sf = p.sfield;
  const unsigned oc = unsigned((y0 + ty) * p.nx + (x0 + tx)) * 8u;  // own column, bytes

  if (tid < CMHD_MAX_RAD) {
    sm.rad[tid] = p.rad_lnT[tid];
    sm.rad[CMHD_MAX_RAD + tid] = p.rad_lnL[tid];
    sm.rad[2 * CMHD_MAX_RAD + tid] = p.rad_slope[tid];
  }

  // this wave's share of the copies of the RK register and of f at the own
  // tile: wave w copies field w, two 16-byte chunks per lane (a 16 x 16 tile
  // row is 8 chunks)
  const int cw = wave;
  unsigned coff[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int ch = m * 64 + (tid & 63);
    coff[m] = unsigned((y0 + ch / 8) * p.nx + x0 + (ch % 8) * 2) * 8u;
  }

  // F of plane kf: the register updates, from LDS only (the right-hand sides,
  // the copied RK register and f), so that it runs while the window waves
  // stage the next plane.  The magnetic waves update A (with the photospheric
  // nudging); the fluid waves add the magnetic terms, apply the boundary
  // terms and update u, ln rho, ln T.
  auto finish = [&](int kf) {
    const long long pl = (kf + NG) * sp;
    const int oo = opaque(o);
    const OwnSrc<Real> own{&sm.Fown[0][0] + oo};
    PointCtx<Real> pc;
    pc.bottom = SOLAR && kf == 0;
    pc.top = SOLAR && kf == p.nz - 1;
    pc.ramp = st.ramp;
    if (mag) {
      Real out[NF];
#pragma unroll
      for (int i = 0; i < 3; ++i) out[AX + i] = sm.QA[i][oo];
      if (SOLAR && kf == 0) {
        pc.ah[0] = Real(ld_u(ah, oc));
        pc.ah[1] = Real(ld_u(ah + sp, oc));
        rhs_boundary_magnetic<Real>(own, pc, p, out);
      }
      // 2N-RK3 update of A in float64
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int fi = AX + i;
        const double r = double(out[fi]);
        const double d = READ_DF ? st.alpha * sm.R[fi][oo] + st.dt * r : st.dt * r;
        if (WRITE_DF) st_u(dF + fi * sf + pl, oc, d);
        st_u(fo + fi * sf + pl, oc, own.v64(fi) + st.beta * d);
      }
    } else {
      Real out[NF];
#pragma unroll
      for (int i = 0; i < 3; ++i) out[UX + i] = sm.Q[i][oo];
      out[LR] = sm.Q[3][oo];
      out[LT] = sm.Q[4][oo];
      {
        Real add[NXCH];
#pragma unroll
        for (int i = 0; i < NXCH; ++i) add[i] = sm.X[i][oo];
        rhs_add_magnetic<Real>(add, out);
      }
      if (SOLAR && kf == 0) {
        pc.uh[0] = Real(ld_u(uh, oc));
        pc.uh[1] = Real(ld_u(uh + sp, oc));
      }
      rhs_boundary_fluid<Real>(own, pc, p, out);
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const int fi = UX + i;
        const double r = double(out[fi]);
        double d = READ_DF ? st.alpha * sm.R[fi][oo] + st.dt * r : st.dt * r;
        double fnew = own.v64(fi) + st.beta * d;
        if (SOLAR) {
          // closed boundary (u_z = 0 at both boundary planes) and the
          // photospheric density held at its initial value ('fg')
          const bool fixz = (fi == UZ) && (kf == 0 || kf == p.nz - 1);
          const bool fixr = (fi == LR) && (kf == 0);
          if (fixz || fixr) {
            d = 0.0;
            fnew = fixr ? p.lnrho0_bot[3] : 0.0;
          }
        }
        if (WRITE_DF) st_u(dF + fi * sf + pl, oc, d);
        st_u(fo + fi * sf + pl, oc, fnew);
      }
    }
  };

  for (int k = kbeg; k < kend; ++k) {
    const long long pl = (k + NG) * sp;
    // ---- F of the previous plane (the window waves stage this one)
    if (k > kbeg) finish(k - 1);
    lds_barrier();     // B1: the plane is staged; the previous plane's F reads are done
    const int oo = opaque(o);   // own column for the direct LDS accesses of this plane
    // ---- the RK register and f of the own tile into LDS, in flight during X
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      unsigned off = coff[m];
      asm volatile("" : "+v"(off));
      if (READ_DF)
        copy16(reinterpret_cast<const char*>(dF + cw * sf + pl) + off, &sm.R[cw][m * 128]);
      copy16(reinterpret_cast<const char*>(f + cw * sf + pl) + off, &sm.Fown[cw][m * 128]);
    }
    // ---- X: D1_x of the xy-mixed fields (with the window waves), the
    // radiative loss on the magnetic waves; the parts of continuity and
    // energy without div u and S:S (and the Newtonian cooling) on the fluid
    // waves
    stencils_dx<Real, NEWTON, false>(sm, tid);
    {
      const int io = opaque(ty * HW + tx), iz = opaque(o);
      const LdsSrc<Real> src{&sm.P[0][0] + io, &sm.Z[0][0] + io, &sm.ZZ[0][0] + iz,
                             &sm.Dx[0][0], p.i60dx, p.i60dy, p.i180dx2, p.i180dy2, 0.0};
      if (mag) {
        sm.Q[5][oo] = rhs_radiation<Real>(src, p, LdsRadTable{sm.rad});
        sm.Q[8][oo] = point_irho<Real>(src);
      } else {
        PointCtx<Real> pc;
        swamp(p, k, pc.w, pc.dw);
        Real nc = Real(0.0);
        if (NEWTON) {
          pc.nc_cz = nc_height_cut(p, k);
          pc.nc_lnT0 = p.nc_tab[p.nc_n + k + NG];
          nc = rhs_newton<Real>(src, p, ParamNcTable{p}, pc);
        }
        Real LRp, LTp, T, icvT;
        rhs_scalars_pre<Real>(src, pc, p, nc, LRp, LTp);
        point_temperature<Real>(src, p, T, icvT);
        sm.Q[3][oo] = LRp;
        sm.Q[4][oo] = LTp;
        sm.Q[6][oo] = T;
        sm.Q[7][oo] = icvT;
      }
    }
    copies_barrier();  // B2: D1_x and the pointwise terms staged, the copies landed

    // ---- R: right-hand side at the own column
    const int io = opaque(ty * HW + tx), ixo = opaque(ty * TX + tx), iz = opaque(o);
    const LdsSrc<Real> src{&sm.P[0][0] + io, &sm.Z[0][0] + io, &sm.ZZ[0][0] + iz,
                           &sm.Dx[0][0] + ixo, p.i60dx, p.i60dy, p.i180dx2, p.i180dy2,
                           p.i60dx * p.i60dy};
    PointCtx<Real> pc;
    swamp(p, k, pc.w, pc.dw);
    if (mag) {
      Real out[NF];
      MagState<Real> m;
      rhs_magnetic<Real>(src, pc, p, out, m);
#pragma unroll
      for (int i = 0; i < 3; ++i) sm.QA[i][oo] = out[AX + i];
      const PointVals<Real> pv{sm.Q[6][oo], sm.Q[8][oo], sm.Q[7][oo]};
      {
        Real add[3];
        rhs_lorentz<Real>(m, pv, add);
#pragma unroll
        for (int i = 0; i < 3; ++i) sm.X[i][oo] = add[i];
      }
      sm.X[3][oo] = rhs_heating<Real>(src, pc, p, m, pv);
    } else {
      Real out[NF], divu, SS;
      const PointVals<Real> pv{sm.Q[6][oo], Real(0.0), sm.Q[7][oo]};
      rhs_momentum<Real>(src, p, pv, out, divu, SS);
#pragma unroll
      for (int i = 0; i < 3; ++i) sm.Q[i][oo] = out[UX + i];
      Real dlr, dlT;
      rhs_scalars_post<Real>(p, pv, sm.Q[3][oo], sm.Q[4][oo], divu, SS, sm.Q[5][oo], dlr,
                             dlT);
      sm.Q[3][oo] = dlr;
      sm.Q[4][oo] = dlT;
    }
    lds_barrier();     // B3: right-hand sides done; the staged plane is free
  }
  finish(kend - 1);
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
hipError_t launch_typed(const KParams& p, const KParams* pg, int stage, const double* f,
                        double* fo, double* dF, const double* uh, const double* ah, StageArgs st,
                        const SubstagePlan& sp, hipStream_t s) {
  TileMap tm{p.nx / TX, p.ny / TY, 8, 4, 0};
  tm.pw = tm.ntx < tm.pw ? tm.ntx : tm.pw;
  tm.ph = tm.nty < tm.ph ? tm.nty : tm.ph;
  // XCD-aware order when the patches split evenly over the 8 XCDs
  tm.xcd = ((tm.ntx / tm.pw) * (tm.nty / tm.ph) * sp.nchunk) % 8 == 0;
  dim3 grid(unsigned(tm.ntx * tm.nty * sp.nchunk));
  if (stage == 0)
    hipLaunchKernelGGL((k_substage<Real, SOLAR, false, true, NEWTON>), grid, dim3(NTB), 0, s, f,
                       fo, dF, uh, ah, p, st, sp.kchunk, tm);
  else if (stage == 1)
    hipLaunchKernelGGL((k_substage<Real, SOLAR, true, true, NEWTON>), grid, dim3(NTB), 0, s, f,
                       fo, dF, uh, ah, p, st, sp.kchunk, tm);
  else
    hipLaunchKernelGGL((k_substage<Real, SOLAR, true, false, NEWTON>), grid, dim3(NTB), 0, s, f,
                       fo, dF, uh, ah, p, st, sp.kchunk, tm);
  return hipGetLastError();
}

// the Newtonian cooling variant is built for the solar (stratified) mode only
template <typename Real>
hipError_t launch_prec(const KParams& p, const KParams* pg, int stage, const double* f,
                       double* fo, double* dF, const double* uh, const double* ah, StageArgs st,
                       const SubstagePlan& sp, hipStream_t s) {
  if (p.solar && p.nc_tau != 0.0)
    return launch_typed<Real, true, true>(p, pg, stage, f, fo, dF, uh, ah, st, sp, s);
  if (p.solar)
    return launch_typed<Real, true, false>(p, pg, stage, f, fo, dF, uh, ah, st, sp, s);
  return launch_typed<Real, false, false>(p, pg, stage, f, fo, dF, uh, ah, st, sp, s);
}

}  // namespace

SubstagePlan plan_substage(const KParams& p) {
  // z chunks so that the grid has about 2048 blocks (8 per CU): on large
  // grids each block marches a long chunk (the 6-plane window prologue is
  // amortised), small grids are cut into short chunks to fill the GPU
  SubstagePlan c;
  const int tiles = (p.nx / TX) * (p.ny / TY);
  int nchunk = (2048 + tiles - 1) / tiles;
  if (nchunk > p.nz) nchunk = p.nz;
  c.kchunk = (p.nz + nchunk - 1) / nchunk;
  c.nchunk = (p.nz + c.kchunk - 1) / c.kchunk;
  return c;
}

hipError_t launch_substage(const KParams& p, const KParams* pg, int prec, int stage,
                           const double* f, double* fo, double* dF, const double* uh,
                           const double* ah, StageArgs st, hipStream_t s) {
  const SubstagePlan sp = plan_substage(p);
  if (prec == CMHD_FP32_SPLIT)
    return launch_prec<float>(p, pg, stage, f, fo, dF, uh, ah, st, sp, s);
  return launch_prec<double>(p, pg, stage, f, fo, dF, uh, ah, st, sp, s);
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
