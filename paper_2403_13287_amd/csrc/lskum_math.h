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

// a / b with one Newton-Raphson step on the hardware reciprocal and no
// correction of the product: within 16 ulp (9.4 measured over quotients
// spanning 60 orders of magnitude; the estimate is good to about 2^-24),
// enough for the limiter's quotient, which only scales an increment, at
// three fewer FP64 operations than lk_div.
__device__ __forceinline__ double lk_div1(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  return a * r;
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
// (paper_2403_13287_amd/fit_poly.py: least squares on Chebyshev nodes in
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

// e^x = 2^k e^r with k = rint(x / ln 2) and r = x - k ln 2 (ln 2 split in a
// 32-bit head, so that k ln2_hi is exact, and a tail; Cody and Waite's
// reduction), |r| <= ln(2)/2;
// e^r = 1 + r + r^2 Q(r), Q of degree 9 fitted on that interval
// (paper_2403_13287_amd/fit_poly.py, relative fit error 4e-18), its
// coefficients in scalar registers as in lk_erf.  The scaling by 2^k
// (v_ldexp) gives 0 below about -745 and +inf above about 709.8; NaN
// stays NaN, and so does -inf (the kernels meet it only in states they
// already flag as non-physical).
__device__ __forceinline__ double lk_exp(double x) {
  constexpr double kLog2e = 1.4426950408889634074;
  constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
  constexpr double kLn2Lo = 1.9082149292705878161e-10;
  const double k = __builtin_rint(x * kLog2e);
  double r = fma(-k, kLn2Hi, x);
  r = fma(-k, kLn2Lo, r);
  double p = fma_sc(2.5024645209649299235e-8, r, 2.7631125446226205028e-7);
  p = fma_sc(p, r, 2.7557507285412289794e-6);
  p = fma_sc(p, r, 2.4801490346235071109e-5);
  p = fma_sc(p, r, 1.984126959711890376e-4);
  p = fma_sc(p, r, 1.3888888946678827123e-3);
  p = fma_sc(p, r, 8.3333333334514329145e-3);
  p = fma_sc(p, r, 4.1666666666516322379e-2);
  p = fma_sc(p, r, 1.6666666666666482434e-1);
  p = fma_sc(p, r, 5.0000000000000127272e-1);
  p = fma(fma(p, r, 1.0), r, 1.0);
  // |k| <= 2000 already gives 0 or +inf; the clamp keeps the conversion
  // to int in range
  return __builtin_amdgcn_ldexp(p, (int)fmin(fmax(k, -2000.0), 2000.0));
}

}  // namespace lskum_math
