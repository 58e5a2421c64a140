// The z-derivative pass of one 2N-RK3 substage: k_zderiv streams the state
// once in z and writes the sixth-order d/dz and d2/dz2 of the 8 fields (16
// slots, [slot][nz][ny][nx], in the precision of the right-hand side), which
// the fused kernel (rhs_rk.hip) stages plane by plane.  A translation unit of
// its own, so that each of the two kernels is compiled with the instruction
// scheduling that suits it.
#include "launch.h"

namespace cmhd {
namespace {

constexpr int NZSLOT = 2 * NF;   // d/dz and d2/dz2 of the 8 fields

// ---------------------------------------------------------------------------
// z derivatives: one thread per (column, field), marching over a chunk of
// planes with the 7-plane window in registers.  STRETCH: the stencils act in
// the plane index and the metric of the non-uniform grid scales them,
// d/dz = c1 S1, d2/dz2 = c2 S2 + c3 S1 (S1, S2 the unscaled stencil sums)
template <typename Real, bool STRETCH>
__global__ __launch_bounds__(256) void k_zderiv(const double* __restrict__ f,
                                                Real* __restrict__ dz, const KParams p,
                                                int kfirst, int klast, int kchunk) {
  const long long sp = p.splane;
  const long long col = blockIdx.x * 256LL + threadIdx.x;
  const int fi = blockIdx.y;
  const int k0 = kfirst + blockIdx.z * kchunk;
  const int k1 = min(k0 + kchunk, klast);
  const long long szs = (long long)p.nz * sp;
  const double* a = f + fi * p.sfield + col;   // array plane j at a[j * sp]
  Real* o1 = dz + fi * szs + col;
  Real* o2 = dz + (NF + fi) * szs + col;
  double w0 = a[(k0 + 0) * sp], w1 = a[(k0 + 1) * sp], w2 = a[(k0 + 2) * sp];
  double w3 = a[(k0 + 3) * sp], w4 = a[(k0 + 4) * sp], w5 = a[(k0 + 5) * sp];
  for (int k = k0; k < k1; ++k) {
    const double w6 = a[(k + 6) * sp];
    double d1, d2;
    if (STRETCH) {
      const double s1 = 45.0 * (w4 - w2) - 9.0 * (w5 - w1) + (w6 - w0);
      const double s2 = -490.0 * w3 + 270.0 * (w4 + w2) - 27.0 * (w5 + w1) + 2.0 * (w6 + w0);
      d1 = s1 * p.ztab[zt_c1(p) + k];
      d2 = s2 * p.ztab[zt_c2(p) + k] + s1 * p.ztab[zt_c3(p) + k];
    } else {
      d1 = (45.0 * (w4 - w2) - 9.0 * (w5 - w1) + (w6 - w0)) * p.i60dz;
      d2 = (-490.0 * w3 + 270.0 * (w4 + w2) - 27.0 * (w5 + w1) + 2.0 * (w6 + w0)) * p.i180dz2;
    }
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

template <typename Real>
hipError_t launch_zderiv_typed(const KParams& p, const double* f, void* dz, int k0, int k1,
                               hipStream_t s) {
  const int kchunk = 32;
  const int nchunk = (k1 - k0 + kchunk - 1) / kchunk;
  dim3 grid(unsigned(p.splane / 256), NF, nchunk);
  if (p.stretched)
    hipLaunchKernelGGL((k_zderiv<Real, true>), grid, dim3(256), 0, s, f, static_cast<Real*>(dz),
                       p, k0, k1, kchunk);
  else
    hipLaunchKernelGGL((k_zderiv<Real, false>), grid, dim3(256), 0, s, f, static_cast<Real*>(dz),
                       p, k0, k1, kchunk);
  return hipGetLastError();
}

}  // namespace

size_t zderiv_bytes(const KParams& p, int prec) {
  const size_t el = prec == CMHD_FP32_SPLIT ? sizeof(float) : sizeof(double);
  return size_t(NZSLOT) * size_t(p.nz) * size_t(p.splane) * el;
}

hipError_t launch_zderiv(const KParams& p, int prec, const double* f, void* dz, int k0, int k1,
                         hipStream_t s) {
  return prec == CMHD_FP32_SPLIT ? launch_zderiv_typed<float>(p, f, dz, k0, k1, s)
                                 : launch_zderiv_typed<double>(p, f, dz, k0, k1, s);
}

}  // namespace cmhd
