// Ghost planes in z and the 2-D Fourier work of the magnetic boundaries.
//
// Solar mode (vertex-centred z, k = 0 photosphere, k = nz-1 top):
//   below (k = -j):  A by the inverted potential field exp(+f_bot |k| j dz)
//                    (Sect. 2.4), u_z antisymmetric (closed, Sect. 2.5),
//                    ln rho = initial profile ('fg'), ln T by the hydrostatic
//                    recursion of eq. (8) read as
//                      ln T(-j) = ln T(-j+1) + ln rho(-j+1) - ln rho(-j)
//                                 - dz g / (R T(-j+1)),
//                    u_x, u_y are state (not touched);
//   above (k = nz-1+j, mirror m = nz-1-j): A by the potential field
//                    exp(-|k| j dz) (eqs. 16-17), u_z antisymmetric, u_x, u_y
//                    symmetric (closed, Sect. 4.1), ln T symmetric (eq. 11),
//                    ln rho(nz-1+j) = ln rho(m) + g (z_{nz-1+j} - z_m)/(R T(nz-1))
//                    (eq. 13 with p = rho R T).
// Periodic mode: plane copies.
//
// Fourier transforms: radix-2 decimation-in-time, one workgroup per 1-D
// transform staged in LDS, float64 throughout; the potential-field ghosts in
// three fused passes (rows forward; per column forward, filter, inverse;
// rows inverse), the other 2-D transforms as rows then columns.  Forward
// transform unnormalised, inverse normalised by 1/(nx ny) in the spectral
// filter.  Because the multipliers are real and even in k, two real
// planes are filtered at once as the real and imaginary parts of one complex
// plane.
#include "launch.h"

namespace cmhd {
namespace {

constexpr double TWO_PI = 6.283185307179586476925286766559;

// ---------------------------------------------------------------------------
// z ghosts
// ---------------------------------------------------------------------------

__global__ void k_fill_periodic_z(const KParams p, double* __restrict__ f) {
  const long long plane = p.splane;
  const long long n = (long long)NF * 2 * NG * plane;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int fi = int(i / (2 * NG * plane));
    const long long r = i - (long long)fi * 2 * NG * plane;
    const int j = int(r / plane);          // 0..5
    const long long col = r - (long long)j * plane;
    double* a = f + fi * p.sfield + col;
    if (j < NG) {
      a[j * plane] = a[(p.nz + j) * plane];                       // below <- top of interior
    } else {
      const int jj = j - NG;
      a[(p.nz + NG + jj) * plane] = a[(NG + jj) * plane];          // above <- bottom of interior
    }
  }
}

__global__ void k_fill_solar_columns(const KParams p, double* __restrict__ f) {
  const long long sp = p.splane;
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < sp;
       col += (long long)gridDim.x * blockDim.x) {
    double* uz = f + UZ * p.sfield + col;
    double* ux = f + UX * p.sfield + col;
    double* uy = f + UY * p.sfield + col;
    double* lr = f + LR * p.sfield + col;
    double* lT = f + LT * p.sfield + col;
    const int kb = NG;                 // array plane of k = 0
    const int kt = NG + p.nz - 1;      // array plane of k = nz-1
#pragma unroll
    for (int j = 1; j <= NG; ++j) {
      uz[(kb - j) * sp] = -uz[(kb + j) * sp];
      uz[(kt + j) * sp] = -uz[(kt - j) * sp];
      ux[(kt + j) * sp] = ux[(kt - j) * sp];
      uy[(kt + j) * sp] = uy[(kt - j) * sp];
      lr[(kb - j) * sp] = p.lnrho0_bot[NG - j];
    }
    // hydrostatic lower temperature ghosts, recursive downward (eq. 8)
#pragma unroll
    for (int j = 1; j <= NG; ++j) {
      const int up = kb - j + 1;
      const double Tup = exp(lT[up * sp]);
      lT[(kb - j) * sp] =
          lT[up * sp] + lr[up * sp] - lr[(kb - j) * sp] - p.dz_lo[j - 1] * p.g_z / (p.R * Tup);
    }
    // symmetric temperature above (eq. 11)
#pragma unroll
    for (int j = 1; j <= NG; ++j) lT[(kt + j) * sp] = lT[(kt - j) * sp];
    if (!p.stretched) {
      // hydrostatic mirror density (eq. 13; symmetric grid distances)
      const double Ttop = exp(lT[kt * sp]);
#pragma unroll
      for (int j = 1; j <= NG; ++j)
        lr[(kt + j) * sp] = lr[(kt - j) * sp] + p.g_z * (2.0 * j * p.dz) / (p.R * Ttop);
    } else {
      // non-uniform grid: the recursion of eq. (15), upward
#pragma unroll
      for (int j = 1; j <= NG; ++j) {
        const double Ta = exp(lT[(kt + j - 1) * sp]), Tb = exp(lT[(kt + j) * sp]);
        lr[(kt + j) * sp] = lr[(kt + j - 1) * sp] + p.dz_hi[j - 1] * 2.0 * p.g_z / (p.R * (Tb + Ta));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 1-D FFT in LDS: one workgroup per transform, length n = 2^logn <= 1024
// ---------------------------------------------------------------------------

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int brev(int t, int logn) {
  return (int)(__brev((unsigned)t) >> (32 - logn));
}

// the twiddles exp(-2 pi i k / n), k < n/2, into LDS (one sincospi per thread)
__device__ __forceinline__ void twiddles(double2* tw, int t, int n) {
  if (t < n / 2) {
    double sn, cs;
    sincospi(2.0 * t / n, &sn, &cs);
    tw[t] = make_double2(cs, -sn);
  }
}

// Radix-2 decimation in time over the n = blockDim.x threads of the block: on
// entry thread t holds element brev(t) of the input, on return element t of
// its transform (sign -1 forward, +1 with INV).  A butterfly's partner
// t ^ half lies in the same wavefront for half < 64 and is exchanged with a
// lane shuffle; the longer stages exchange through buf.  The stage of length
// len uses the twiddle k = pos n / len.  Ends with buf free for reuse.
template <bool INV>
__device__ __forceinline__ double2 fft_stages(double2 v, int t, int n, const double2* tw,
                                              double2* buf) {
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1;
    double2 o;
    if (half < 64) {
      o.x = __shfl_xor(v.x, half);
      o.y = __shfl_xor(v.y, half);
    } else {
      buf[t] = v;
      __syncthreads();
      o = buf[t ^ half];
      __syncthreads();
    }
    const int pos = t & (half - 1);
    double2 w = tw[pos * (n / len)];
    if (INV) w.y = -w.y;
    // lower element t: a + w b with b = o; upper element: a - w b with a = o, b = v
    if ((t & half) == 0) {
      const double2 bb = cmul(o, w);
      v = make_double2(v.x + bb.x, v.y + bb.y);
    } else {
      const double2 bb = cmul(v, w);
      v = make_double2(o.x - bb.x, o.y - bb.y);
    }
  }
  return v;
}

// The same stages for M transforms of one block in lockstep (element t of
// each in thread t): one barrier pair and one twiddle read per stage serve
// all of them.  buf holds M * n elements.
template <bool INV, int M>
__device__ __forceinline__ void fft_stages_m(double2 (&v)[M], int t, int n, const double2* tw,
                                             double2* buf) {
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1;
    double2 o[M];
    if (half < 64) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        o[m].x = __shfl_xor(v[m].x, half);
        o[m].y = __shfl_xor(v[m].y, half);
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) buf[m * n + t] = v[m];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < M; ++m) o[m] = buf[m * n + (t ^ half)];
      __syncthreads();
    }
    const int pos = t & (half - 1);
    double2 w = tw[pos * (n / len)];
    if (INV) w.y = -w.y;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if ((t & half) == 0) {
        const double2 bb = cmul(o[m], w);
        v[m] = make_double2(v[m].x + bb.x, v[m].y + bb.y);
      } else {
        const double2 bb = cmul(v[m], w);
        v[m] = make_double2(o[m].x - bb.x, o[m].y - bb.y);
      }
    }
  }
}

// Blocks are dispatched round-robin to the 8 XCDs, each with its own L2.  A
// column transform touches 16 bytes of every row, so the 8 columns that share
// a 128-byte line are given to blocks on one XCD: block id -> transform index
// with each XCD taking a contiguous range (nblocks a multiple of 8).
__device__ __forceinline__ long long xcd_order(long long id, long long nblocks) {
  if (nblocks & 7) return id;
  return (id & 7) * (nblocks >> 3) + (id >> 3);
}

// transform b: elements at base(b) + j*stride, j = 0..n-1, where
// base(b) = (b / inner) * outer + (b % inner) * istride; XCD-ordered when
// the transforms are strided columns
__global__ __launch_bounds__(1024) void k_fft1d(double2* __restrict__ data, int n, int logn,
                                                long long stride, int inner, long long outer,
                                                long long istride, double sign) {
  __shared__ double2 buf[1024];
  __shared__ double2 tw[512];
  const long long b = stride == 1 ? (long long)blockIdx.x : xcd_order(blockIdx.x, gridDim.x);
  const long long base = (b / inner) * outer + (b % inner) * istride;
  const int t = threadIdx.x;
  double2 v = data[base + brev(t, logn) * stride];
  twiddles(tw, t, n);
  __syncthreads();
  v = sign > 0.0 ? fft_stages<true>(v, t, n, tw, buf) : fft_stages<false>(v, t, n, tw, buf);
  data[base + t * stride] = v;
}

}  // namespace

// forward (sign -1) or inverse (+1) 2-D transform of nplanes planes [ny][nx]
hipError_t fft2d(const KParams& p, double2* d, int nplanes, double sign, hipStream_t s) {
  const int nx = p.nx, ny = p.ny;
  const long long plane = (long long)nx * ny;
  // rows: transform b = (plane, row); contiguous; one thread per element
  hipLaunchKernelGGL(k_fft1d, dim3(nplanes * ny), dim3(nx), 0, s, d, nx, ilog2(nx), 1LL, 1,
                     (long long)nx, 0LL, sign);
  // columns: transform b = (plane, column); stride nx
  hipLaunchKernelGGL(k_fft1d, dim3(nplanes * nx), dim3(ny), 0, s, d, ny, ilog2(ny),
                     (long long)nx, nx, plane, 1LL, sign);
  return hipGetLastError();
}

namespace {

// The potential-field ghosts of A in three passes over the complex planes
// q = 0: Ax + i Ay (bottom), 1: Az (bottom), 2: Ax + i Ay (top), 3: Az (top):
//   rows     the boundary rows of f transformed along x into S[q] (the two
//            planes of one boundary and row index in lockstep);
//   columns  each column of S[q] transformed along y, multiplied by the
//            filter of ghost layer j and transformed back along y, into
//            T[3q + j-1] (one forward and three inverse transforms per block,
//            the three in lockstep);
//   rows     the three rows of T[3q .. 3q+2] at one row index transformed
//            back along x in lockstep and written into the ghost planes of f.
// The inverse 2-D transform takes its columns first: the two 1-D passes
// commute.

__device__ __forceinline__ long long pf_plane(const KParams& p, int q) {
  return (q < 2 ? NG : NG + p.nz - 1) * p.splane;
}

// block (boundary, row) of 2 * ny, nx threads: the two planes q = 2 side,
// 2 side + 1 (A_x + i A_y and A_z of the bottom or top plane) of one row
// index in lockstep
__global__ __launch_bounds__(1024) void k_pf_rows_fwd(const KParams p,
                                                      const double* __restrict__ f,
                                                      double2* __restrict__ S) {
  extern __shared__ double2 dyn[];   // [2 * n] exchange | [n/2] twiddles
  double2* buf = dyn;
  double2* tw = dyn + 2 * p.nx;
  const int side = blockIdx.x / p.ny, row = blockIdx.x - side * p.ny;
  const int t = threadIdx.x, n = p.nx;
  const long long o = pf_plane(p, 2 * side) + (long long)row * n + brev(t, ilog2(n));
  double2 v[2] = {make_double2(f[AX * p.sfield + o], f[AY * p.sfield + o]),
                  make_double2(f[AZ * p.sfield + o], 0.0)};
  twiddles(tw, t, n);
  __syncthreads();
  fft_stages_m<false, 2>(v, t, n, tw, buf);
#pragma unroll
  for (int m = 0; m < 2; ++m) S[(2 * side + m) * p.splane + (long long)row * n + t] = v[m];
}

// T[3q + j-1] = S[q] exp(-|k| d_qj) / (nx ny) along each column, with
// d = -f_bot (z(0) - z(-j)) below (the contrast grows with depth, Sect. 2.4)
// and d = z(nz-1+j) - z(nz-1) above (eq. 17).  Block (q, column) of 4 * nx,
// XCD-ordered, ny threads.
__global__ __launch_bounds__(1024) void k_pf_columns(const KParams p,
                                                     const double2* __restrict__ S,
                                                     double2* __restrict__ T) {
  extern __shared__ double2 dyn[];   // [NG * n] exchange | [n/2] twiddles
  double2* buf = dyn;
  double2* tw = dyn + NG * p.ny;
  const int b = int(xcd_order(blockIdx.x, gridDim.x));
  const int q = b / p.nx, col = b - q * p.nx;
  const int t = threadIdx.x, n = p.ny, logn = ilog2(n);
  const long long sp = p.splane;
  const double2 v0 = S[q * sp + (long long)brev(t, logn) * p.nx + col];
  twiddles(tw, t, n);
  __syncthreads();
  const double2 v = fft_stages<false>(v0, t, n, tw, buf);
  const double k = kabs(p, col, t);
  const double* dist = p.pf_dist[q < 2 ? 0 : 1];
  const double inv_n = 1.0 / double(sp);
  double2 u[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const double fac = exp(-k * dist[j]) * inv_n;
    buf[j * n + t] = make_double2(v.x * fac, v.y * fac);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NG; ++j) u[j] = buf[j * n + brev(t, logn)];
  __syncthreads();
  fft_stages_m<true, NG>(u, t, n, tw, buf);
#pragma unroll
  for (int j = 0; j < NG; ++j) T[(q * NG + j) * sp + (long long)t * p.nx + col] = u[j];
}

// block (q, row) of 4 * ny, nx threads: the three ghost layers j = 1..3
// below (q < 2) or above, transformed in lockstep
__global__ __launch_bounds__(1024) void k_pf_rows_inv(const KParams p,
                                                      const double2* __restrict__ T,
                                                      double* __restrict__ f) {
  extern __shared__ double2 dyn[];   // [NG * n] exchange | [n/2] twiddles
  double2* buf = dyn;
  double2* tw = dyn + NG * p.nx;
  const int q = blockIdx.x / p.ny, row = blockIdx.x - q * p.ny;
  const int t = threadIdx.x, n = p.nx;
  const long long c = (long long)row * n + brev(t, ilog2(n));
  double2 u[NG];
#pragma unroll
  for (int j = 0; j < NG; ++j) u[j] = T[(q * NG + j) * p.splane + c];
  twiddles(tw, t, n);
  __syncthreads();
  fft_stages_m<true, NG>(u, t, n, tw, buf);
#pragma unroll
  for (int j = 1; j <= NG; ++j) {
    const long long o =
        (q < 2 ? NG - j : NG + p.nz - 1 + j) * p.splane + (long long)row * n + t;
    if (q & 1) {
      f[AZ * p.sfield + o] = u[j - 1].x;
    } else {
      f[AX * p.sfield + o] = u[j - 1].x;
      f[AY * p.sfield + o] = u[j - 1].y;
    }
  }
}

// A_h* from B_z (eq. 7): A^_x + i A^_y = (k_x + i k_y) B^_z / k^2, zero mean
// and Nyquist rows/columns, normalised for the inverse transform
__global__ void k_pack_real(const KParams p, const double* __restrict__ a,
                            double2* __restrict__ S) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p.splane;
       i += (long long)gridDim.x * blockDim.x)
    S[i] = make_double2(a[i], 0.0);
}

__global__ void k_ah_spectrum(const KParams p, double2* __restrict__ S) {
  const double inv_n = 1.0 / double(p.splane);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p.splane;
       i += (long long)gridDim.x * blockDim.x) {
    const int iy = int(i / p.nx), ix = int(i - (long long)iy * p.nx);
    const int mx = ix < p.nx / 2 ? ix : ix - p.nx;
    const int my = iy < p.ny / 2 ? iy : iy - p.ny;
    if ((mx == 0 && my == 0) || ix == p.nx / 2 || iy == p.ny / 2) {
      S[i] = make_double2(0.0, 0.0);
      continue;
    }
    const double kx = TWO_PI * mx / p.Lx, ky = TWO_PI * my / p.Ly;
    const double ik2 = inv_n / (kx * kx + ky * ky);
    const double2 b = S[i];
    // (kx + i ky) * b
    S[i] = make_double2((kx * b.x - ky * b.y) * ik2, (kx * b.y + ky * b.x) * ik2);
  }
}

__global__ void k_unpack_ah(const KParams p, const double2* __restrict__ S,
                            double* __restrict__ ah) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p.splane;
       i += (long long)gridDim.x * blockDim.x) {
    ah[i] = S[i].x;
    ah[p.splane + i] = S[i].y;
  }
}

// ---------------------------------------------------------------------------
// reductions: CFL maxima, finiteness, net flux
// ---------------------------------------------------------------------------

// atomic max of non-negative doubles through their bit patterns (monotone)
__device__ __forceinline__ void atomic_max_pos(unsigned long long* a, double v) {
  atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double d1col(const double* a, long long s) {
  return 45.0 * (a[s] - a[-s]) - 9.0 * (a[2 * s] - a[-2 * s]) + (a[3 * s] - a[-3 * s]);
}

__device__ __forceinline__ long long wrapx(const KParams& p, long long col, int dx) {
  const int y = int(col / p.nx);
  int x = int(col - (long long)y * p.nx) + dx;
  x += x < 0 ? p.nx : 0;
  x -= x >= p.nx ? p.nx : 0;
  return (long long)y * p.nx + x;
}
__device__ __forceinline__ long long wrapy(const KParams& p, long long col, int dy) {
  int y = int(col / p.nx);
  const int x = int(col - (long long)y * p.nx);
  y += dy;
  y += y < 0 ? p.ny : 0;
  y -= y >= p.ny ? p.ny : 0;
  return (long long)y * p.nx + x;
}

// first derivative along x or y of field fi at plane-array index kz, column col
__device__ double d1xy(const KParams& p, const double* f, int fi, int kz, long long col,
                       int axis) {
  const double* a = f + fi * p.sfield + (long long)kz * p.splane;
  double acc = 0.0;
  const double cf[3] = {45.0, -9.0, 1.0};
#pragma unroll
  for (int m = 1; m <= 3; ++m) {
    const long long cp = axis == 0 ? wrapx(p, col, m) : wrapy(p, col, m);
    const long long cm = axis == 0 ? wrapx(p, col, -m) : wrapy(p, col, -m);
    acc += cf[m - 1] * (a[cp] - a[cm]);
  }
  return acc * (axis == 0 ? p.i60dx : p.i60dy);
}

// One block per (y, z) row of the interior, threads along x: the periodic
// neighbours are found by comparison, with no integer division per zone.
__global__ void k_cfl(const KParams p, const double* __restrict__ f,
                      unsigned long long* __restrict__ out3) {
  __shared__ double red[3][256];
  double ms = 0.0, md = 0.0, mr = 0.0;
  const long long nrows = (long long)p.nz * p.ny;
  for (long long row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int k = int(row / p.ny), y = int(row - (long long)k * p.ny);
    const int kz = k + NG;
    const long long pl = (long long)kz * p.splane;
    auto wy = [&](int d) { return y + d < 0 ? y + d + p.ny : (y + d >= p.ny ? y + d - p.ny : y + d); };
    const long long ym1 = (long long)wy(-1) * p.nx, ym2 = (long long)wy(-2) * p.nx,
                    ym3 = (long long)wy(-3) * p.nx, yp1 = (long long)wy(1) * p.nx,
                    yp2 = (long long)wy(2) * p.nx, yp3 = (long long)wy(3) * p.nx;
    const double mz = p.stretched ? p.ztab[zt_c1(p) + k] : p.i60dz;
    double w = 0.0;
    if (p.solar) {
      const double z = zk(p, k);
      double s = (z - p.z_s) / (p.z_t - p.z_s);
      s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
      w = s * s * (3.0 - 2.0 * s);
    }
    const double dl = p.stretched ? fmin(p.dxy_min, p.ztab[zt_zp(p) + k]) : 1.0;
    for (int x = threadIdx.x; x < p.nx; x += blockDim.x) {
      const long long o = pl + (long long)y * p.nx + x;
      // x and y first derivatives by the sixth-order stencil, wrapped
      auto wx = [&](int d) { return x + d < 0 ? x + d + p.nx : (x + d >= p.nx ? x + d - p.nx : x + d); };
      const int xm1 = wx(-1), xm2 = wx(-2), xm3 = wx(-3), xp1 = wx(1), xp2 = wx(2), xp3 = wx(3);
      auto dx = [&](int fi) {
        const double* a = f + fi * p.sfield + pl + (long long)y * p.nx;
        return (45.0 * (a[xp1] - a[xm1]) - 9.0 * (a[xp2] - a[xm2]) + (a[xp3] - a[xm3])) * p.i60dx;
      };
      auto dy = [&](int fi) {
        const double* a = f + fi * p.sfield + pl + x;
        return (45.0 * (a[yp1] - a[ym1]) - 9.0 * (a[yp2] - a[ym2]) + (a[yp3] - a[ym3])) * p.i60dy;
      };
      const double dAz_dy = dy(AZ), dAz_dx = dx(AZ);
      const double dAy_dx = dx(AY), dAx_dy = dy(AX);
      const double dAy_dz = d1col(f + AY * p.sfield + o, p.splane) * mz;
      const double dAx_dz = d1col(f + AX * p.sfield + o, p.splane) * mz;
      const double Bx = dAz_dy - dAy_dz + p.Bext[0];
      const double By = dAx_dz - dAz_dx + p.Bext[1];
      const double Bz = dAy_dx - dAx_dy + p.Bext[2];
      const double ux = f[UX * p.sfield + o], uy = f[UY * p.sfield + o], uz = f[UZ * p.sfield + o];
      const double lr = f[LR * p.sfield + o], lT = f[LT * p.sfield + o];
      const double rho = exp(lr), T = exp(lT);
      const double B2 = Bx * Bx + By * By + Bz * Bz;
      const double cf = sqrt(p.gamma * p.R * T + B2 / (p.mu0 * rho));
      double spd = sqrt(ux * ux + uy * uy + uz * uz) + cf;
      double D = p.nu;
      D = fmax(D, p.eta + p.eta_s * w);
      D = fmax(D, p.D_rho + p.chi_rho * w);
      D = fmax(D, p.chi_s * w);
      D = fmax(D, p.kappa0 * exp(2.5 * lT) / (rho * p.cv));
      if (p.stretched) {
        // non-uniform grid: rates per unit of the plane's own spacing
        spd = spd / dl;
        D = D / (dl * dl);
      }
      double rate = 0.0;
      if (p.n_rad > 0 && lT > p.lnT_rad_lo) {
        int seg = 0;
        for (int j = 1; j < p.n_rad - 1; ++j) seg = (lT >= p.rad_lnT[j]) ? j : seg;
        double lnL;
        if (lT < p.rad_lnT[0])
          lnL = p.rad_lnL[0];
        else if (lT >= p.rad_lnT[p.n_rad - 1])
          lnL = p.rad_lnL[p.n_rad - 1];
        else
          lnL = p.rad_lnL[seg] + p.rad_slope[seg] * (lT - p.rad_lnT[seg]);
        double wc = 1.0;
        if (lT < p.lnT_rad_hi) {
          const double s = (lT - p.lnT_rad_lo) * p.inv_dlnT_rad;
          wc = s * s * (3.0 - 2.0 * s);
        }
        rate = exp(lr + lnL - lT) * wc / p.cv;   // Q_rad / (rho c_v T)
      }
      // NaN propagates: fmax would drop it, so test explicitly
      ms = (spd > ms || spd != spd) ? spd : ms;
      md = (D > md || D != D) ? D : md;
      mr = (rate > mr || rate != rate) ? rate : mr;
    }
  }
  red[0][threadIdx.x] = ms;
  red[1][threadIdx.x] = md;
  red[2][threadIdx.x] = mr;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double a = red[q][threadIdx.x], b = red[q][threadIdx.x + s];
        red[q][threadIdx.x] = (b > a || b != b) ? b : a;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) atomic_max_pos(&out3[threadIdx.x], red[threadIdx.x][0]);
}

__global__ void k_zero_u64(unsigned long long* a, int n) {
  if ((int)threadIdx.x < n) a[threadIdx.x] = 0ULL;
}

__global__ void k_bz_plane(const KParams p, const double* __restrict__ f, int k0, double a,
                           double* __restrict__ dst) {
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < p.splane;
       col += (long long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int q = 0; q < 2; ++q) {
      const double wq = q == 0 ? 1.0 - a : a;
      if (wq == 0.0) continue;
      const int kz = k0 + q + NG;
      acc += wq * (d1xy(p, f, AY, kz, col, 0) - d1xy(p, f, AX, kz, col, 1));
    }
    dst[col] = acc + p.Bext[2];
  }
}

__global__ void k_finite(const KParams p, const double* __restrict__ f, int* flag) {
  const long long n = (long long)NF * p.nz * p.splane;
  const long long per = (long long)p.nz * p.splane;
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int fi = int(i / per);
    const long long r = i - fi * per;
    const double v = f[fi * p.sfield + NG * p.splane + r];
    bad |= !isfinite(v);
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void k_sum_abs(const KParams p, const double* __restrict__ a, double* out2) {
  __shared__ double s1[256], s2[256];
  double x1 = 0.0, x2 = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < p.splane;
       i += (long long)gridDim.x * blockDim.x) {
    x1 += a[i];
    x2 += fabs(a[i]);
  }
  s1[threadIdx.x] = x1;
  s2[threadIdx.x] = x2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s1[threadIdx.x] += s1[threadIdx.x + s];
      s2[threadIdx.x] += s2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out2[0], s1[0]);
    atomicAdd(&out2[1], s2[0]);
  }
}

// nudging target between two driver snapshots: u0 + w (u1 - u0)
__global__ void k_driver_interp(long long n, const double* __restrict__ u0,
                                const double* __restrict__ u1, double w,
                                double* __restrict__ uh) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    uh[i] = u0[i] + w * (u1[i] - u0[i]);
}

int grid_for(long long n) {
  long long b = (n + 255) / 256;
  return int(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

hipError_t launch_fill_periodic_z(const KParams& p, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_periodic_z, dim3(grid_for((long long)NF * 2 * NG * p.splane)),
                     dim3(256), 0, s, p, f);
  return hipGetLastError();
}

hipError_t launch_fill_solar_columns(const KParams& p, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_solar_columns, dim3(grid_for(p.splane)), dim3(256), 0, s, p, f);
  return hipGetLastError();
}

hipError_t launch_potential_ghosts(const KParams& p, double* f, double2* scratch,
                                   hipStream_t s) {
  double2* S = scratch;                 // 4 planes
  double2* T = scratch + 4 * p.splane;  // 12 planes
  hipLaunchKernelGGL(k_pf_rows_fwd, dim3(2 * p.ny), dim3(p.nx),
                     (2 * p.nx + p.nx / 2) * sizeof(double2), s, p, f, S);
  hipLaunchKernelGGL(k_pf_columns, dim3(4 * p.nx), dim3(p.ny),
                     (NG * p.ny + p.ny / 2) * sizeof(double2), s, p, S, T);
  hipLaunchKernelGGL(k_pf_rows_inv, dim3(4 * p.ny), dim3(p.nx),
                     (NG * p.nx + p.nx / 2) * sizeof(double2), s, p, T, f);
  return hipGetLastError();
}

hipError_t launch_ah_from_bz(const KParams& p, const double* bz, double* ah, double2* scratch,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_pack_real, dim3(grid_for(p.splane)), dim3(256), 0, s, p, bz, scratch);
  hipError_t e = fft2d(p, scratch, 1, -1.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ah_spectrum, dim3(grid_for(p.splane)), dim3(256), 0, s, p, scratch);
  e = fft2d(p, scratch, 1, +1.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpack_ah, dim3(grid_for(p.splane)), dim3(256), 0, s, p, scratch, ah);
  return hipGetLastError();
}

hipError_t launch_cfl_max(const KParams& p, const double* f, unsigned long long* out3,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, out3, 3);
  const long long rows = (long long)p.nz * p.ny;
  hipLaunchKernelGGL(k_cfl, dim3(unsigned(rows < 65536 ? rows : 65536)), dim3(256), 0, s, p, f,
                     out3);
  return hipGetLastError();
}

hipError_t launch_bz_plane_k(const KParams& p, const double* f, int k0, double a, double* dst,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_bz_plane, dim3(grid_for(p.splane)), dim3(256), 0, s, p, f, k0, a, dst);
  return hipGetLastError();
}

hipError_t launch_bz_plane(const KParams& p, const double* f, double zq, double* dst,
                           hipStream_t s) {
  const double kf = (zq - p.z0) / p.dz;
  int k0 = int(floor(kf));
  double a = kf - k0;
  if (k0 >= p.nz - 1) {
    k0 = p.nz - 2;
    a = 1.0;
  }
  hipLaunchKernelGGL(k_bz_plane, dim3(grid_for(p.splane)), dim3(256), 0, s, p, f, k0, a, dst);
  return hipGetLastError();
}

hipError_t launch_finite_check(const KParams& p, const double* f, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_finite, dim3(grid_for((long long)NF * p.nz * p.splane)), dim3(256), 0, s,
                     p, f, flag);
  return hipGetLastError();
}

hipError_t launch_driver_interp(const KParams& p, const double* u0, const double* u1, double w,
                                double* uh, hipStream_t s) {
  const long long n = 2 * p.splane;
  hipLaunchKernelGGL(k_driver_interp, dim3(grid_for(n)), dim3(256), 0, s, n, u0, u1, w, uh);
  return hipGetLastError();
}

hipError_t launch_sum_abs(const KParams& p, const double* plane, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_abs, dim3(grid_for(p.splane)), dim3(256), 0, s, p, plane, out2);
  return hipGetLastError();
}

}  // namespace cmhd
