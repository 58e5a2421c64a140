// The 72 pointwise inputs of the right-hand side at one zone (values, first
// derivatives, the second derivatives the equations use, lap ln rho), in a
// fixed slot order shared by the forward kernel (which gathers them into
// registers) and the tangent/adjoint kernels (which hold them in a buffer).
#pragma once

#include "cmhd_internal.h"

namespace cmhd {

constexpr int NQ = 72;
__host__ __device__ constexpr int q_v(int f) { return f; }
__host__ __device__ constexpr int q_d(int f, int d) { return 8 + 3 * f + d; }
constexpr int Q_LAPR = 71;
// slot of the second derivative (Hessian slot s: xx yy zz xy xz yz) of field
// f, or -1 where the equations do not use it
__host__ __device__ constexpr int q_h(int f, int s) {
  return f <= AZ ? 32 + 6 * f + s
       : f <= UZ ? (s <= 2 ? 50 + 5 * (f - UX) + s
                   // mixed slots of grad div u: u_x xy xz, u_y xy yz, u_z xz yz
                   : f == UX ? (s == 3 ? 53 : (s == 4 ? 54 : -1))
                   : f == UY ? (s == 3 ? 58 : (s == 5 ? 59 : -1))
                             : (s == 4 ? 63 : (s == 5 ? 64 : -1)))
       : f == LT ? 65 + s
                 : -1;
}
static_assert(q_h(LT, 5) == 70 && Q_LAPR == NQ - 1, "slot layout");

}  // namespace cmhd
