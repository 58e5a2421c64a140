// Forward-mode dual numbers (value + one tangent) for the tangent-linear and
// adjoint kernels: evaluating the pointwise right-hand side program on duals
// gives its directional derivative exactly (to round-off).
#pragma once

#include <hip/hip_runtime.h>

namespace cmhd {

struct Dual {
  double v, d;
  __host__ __device__ Dual() : v(0.0), d(0.0) {}
  __host__ __device__ Dual(double a) : v(a), d(0.0) {}
  __host__ __device__ Dual(double a, double b) : v(a), d(b) {}
};

__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) {
  return Dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual s_exp(Dual a) {
  const double e = exp(a.v);
  return Dual(e, e * a.d);
}
__device__ __forceinline__ Dual s_sqrt(Dual a) {
  const double r = sqrt(a.v);
  return Dual(r, a.d / (2.0 * r));
}
__device__ __forceinline__ Dual s_rsqrt(Dual a) { return Dual(1.0) / s_sqrt(a); }
__device__ __forceinline__ Dual s_sin(Dual a) { return Dual(sin(a.v), cos(a.v) * a.d); }
__device__ __forceinline__ double value_of(Dual a) { return a.v; }

}  // namespace cmhd
