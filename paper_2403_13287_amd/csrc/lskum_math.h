// lskum_math.h -- FP64 helpers for the flux kernel.
//
// lk_div and lk_rsqrt refine the hardware reciprocal / reciprocal square
// root estimates by Newton-Raphson steps (<= 2 ulp for the positive,
// normal arguments the sweep passes: limiter denominators, beta, squared
// edge lengths).  They skip the special-case handling of the general
// library versions, which the sweep never needs.
//
// lk_erf evaluates its polynomial with the coefficients in scalar
// registers: the flux kernel calls erf four times per edge, and the device
// library's erf, inlined there, has its coefficients hoisted into vector
// registers for the whole neighbour loop (about 20 VGPRs, and a register
// copy before every two-address FMA of the Horner steps).
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

// a * b + c with c, a compile-time constant, read from a scalar register
// pair (one scalar operand per vector instruction is allowed), so that the
// compiler materialises it with scalar moves instead of holding it in
// vector registers.
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// erf(x).  |x| < 1: x P(x^2), P of degree 11 fitted to erf(x)/x on [0, 1]
// (paper_2403_13287_amd/fit_erf.py: least squares on Chebyshev nodes in
// 50-digit arithmetic, relative fit error 2e-17); otherwise (and for NaN)
// the device library's erf.  The flux kernel's arguments S = u_d sqrt(beta)
// are mostly below 1 in magnitude (|S| = 0.84 times the directional Mach
// number).
__device__ __forceinline__ double lk_erf(double x) {
  if (!(fabs(x) < 1.0)) return erf(x);
  const double t = x * x;
  double p = fma_sc(-7.7768291373628105931e-10, t, 1.3709519207384054734e-8);
  p = fma_sc(p, t, -1.6205964194101387582e-7);
  p = fma_sc(p, t, 1.6447084274239356277e-6);
  p = fma_sc(p, t, -1.4924708324571507839e-5);
  p = fma_sc(p, t, 1.2055293361789940774e-4);
  p = fma_sc(p, t, -8.5483259218328840198e-4);
  p = fma_sc(p, t, 5.2239776059559766634e-3);
  p = fma_sc(p, t, -2.6866170643090833844e-2);
  p = fma_sc(p, t, 1.1283791670944049985e-1);
  p = fma_sc(p, t, -3.7612638903183516095e-1);
  p = fma_sc(p, t, 1.1283791670955125655);
  return x * p;
}

}  // namespace lskum_math
