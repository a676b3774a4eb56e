// Lagrange weights of the closest-point extension (eq. interp-stencil).
// Cubic: nodes at offsets -1, 0, 1, 2 from floor(y/h), query at fraction t
// in [0,1).
// This is the product form of the Lagrange basis; the barycentric form the
// paper cites is the same polynomial.
#pragma once

#include <hip/hip_runtime.h>

namespace cpm {

// With q = t (t - 1) and (t + 1)(t - 2) = q - 2, each weight is one of these
// two quadratics times a linear factor written as t c + d (10 operations,
// all multiply-adds or products, instead of 15).
template <class T>
__device__ __forceinline__ void lagrange4(T t, T w[4]) {
  const T sixth = T(1) / T(6), third = T(1) / T(3);
  const T q = t * t - t;
  const T q2 = q - T(2);
  w[0] = q * (t * (-sixth) + third);
  w[1] = q2 * (t * T(0.5) - T(0.5));
  w[2] = q2 * (t * T(-0.5));
  w[3] = q * (t * sixth + sixth);
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
