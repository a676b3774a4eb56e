// Cubic Lagrange weights of the closest-point extension (eq. interp-stencil):
// nodes at offsets -1, 0, 1, 2 from floor(y/h), query at fraction t in [0,1).
// This is the product form of the Lagrange basis; the barycentric form the
// paper cites is the same polynomial.
#pragma once

#include <hip/hip_runtime.h>

namespace cpm {

template <class T>
__device__ __forceinline__ void lagrange4(T t, T w[4]) {
  const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
  const T sixth = T(1) / T(6);
  w[0] = -(t * tm1 * tm2) * sixth;
  w[1] = (tp1 * tm1 * tm2) * T(0.5);
  w[2] = -(tp1 * t * tm2) * T(0.5);
  w[3] = (tp1 * t * tm1) * sixth;
}

}  // namespace cpm
