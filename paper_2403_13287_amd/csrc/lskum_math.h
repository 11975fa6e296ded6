// lskum_math.h -- FP64 helpers for the flux kernel.
//
// lk_div and lk_rsqrt refine the hardware reciprocal / reciprocal square
// root estimates by Newton-Raphson steps (<= 2 ulp for the positive,
// normal arguments the sweep passes: limiter denominators, beta, squared
// edge lengths).  They skip the special-case handling of the general
// library versions, which the sweep never needs.
#pragma once

#include <hip/hip_runtime.h>

namespace lskum_math {

__device__ __forceinline__ double lk_div(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  double q = a * r;
  const double res = fma(-b, q, a);
  return fma(r, res, q);
}

__device__ __forceinline__ double lk_rsqrt(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h, r * r, 0.5);
  r = fma(r, e, r);
  e = fma(-h, r * r, 0.5);
  return fma(r, e, r);
}

}  // namespace lskum_math
