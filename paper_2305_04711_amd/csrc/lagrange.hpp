// Lagrange weights of the closest-point extension (eq. interp-stencil).
// Cubic: nodes at offsets -1, 0, 1, 2 from floor(y/h), query at fraction t
// in [0,1).
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

// Quadratic Lagrange weights (p = 2) on nodes -1, 0, 1 relative to the
// nearest node, query at fraction t in [-1/2, 1/2), in a 4-wide vector whose
// last weight is 0 (the tile kernels keep their cubic layout).
template <class T>
__device__ __forceinline__ void lagrange3(T t, T w[4]) {
  const T half = T(0.5);
  w[0] = (t * (t - T(1))) * half;
  w[1] = (T(1) - t) * (T(1) + t);
  w[2] = (t * (t + T(1))) * half;
  w[3] = T(0);
}

template <class T>
__device__ __forceinline__ void lagrange_p(int p, T t, T w[4]) {
  if (p == 3) lagrange4<T>(t, w);
  else lagrange3<T>(t, w);
}

}  // namespace cpm
