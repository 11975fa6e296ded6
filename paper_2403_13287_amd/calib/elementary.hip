// elementary.hip -- calibration kernels for the roofline report.
//
// Each kernel evaluates one FP64 elementary function of the device math
// library once per element over an input array (inputs drawn by the caller
// from the ranges the sweep meets).  Under rocprofv3 the FP64 counters of
// these kernels give the FP64 operations one call costs (FMA = 2), which
// weights the elementary functions in the flux kernel's algorithmic
// operation count.  Not part of the sweep.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../csrc/lskum_math.h"

namespace {

template <int F>
__global__ void __launch_bounds__(256) k_elem(int64_t n, const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i];
  double r;
  if constexpr (F == 0) r = a;
  if constexpr (F == 1) r = exp(a);
  if constexpr (F == 2) r = erf(a);
  if constexpr (F == 3) r = log(a);
  if constexpr (F == 4) r = sqrt(a);
  if constexpr (F == 5) r = rsqrt(a);
  if constexpr (F == 6) r = y[i] / a;
  // the sweep's own versions (lskum_math.h)
  if constexpr (F == 9) r = lskum_math::lk_div(y[i], a);
  if constexpr (F == 10) r = lskum_math::lk_rsqrt(a);
  if constexpr (F == 11) r = lskum_math::lk_erf(a);
  if constexpr (F == 12) r = lskum_math::lk_exp(a);
  if constexpr (F == 13) r = lskum_math::lk_div1(y[i], a);
  out[i] = r;
}

}  // namespace

extern "C" {

// fn: 0 copy (baseline), 1 exp, 2 erf, 3 log, 4 sqrt, 5 rsqrt, 6 divide
// y[i] / x[i]; the sweep's versions: 9 lk_div y[i] / x[i], 10 lk_rsqrt,
// 11 lk_erf, 12 lk_exp, 13 lk_div1 y[i] / x[i].  x, y, out: device arrays of n doubles.  Returns 0, or -1 for
// a bad argument, -3 for a failed launch.
int lskum_calib_elementary(int fn, int64_t n, const double *x, const double *y, double *out,
                           void *stream) {
  if (n <= 0 || !x || !out || ((fn == 6 || fn == 9 || fn == 13) && !y)) return -1;
  const dim3 grid((unsigned)((n + 255) / 256));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  switch (fn) {
    case 0: k_elem<0><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 1: k_elem<1><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 2: k_elem<2><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 3: k_elem<3><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 4: k_elem<4><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 5: k_elem<5><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 6: k_elem<6><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 9: k_elem<9><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 10: k_elem<10><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 11: k_elem<11><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 12: k_elem<12><<<grid, 256, 0, s>>>(n, x, y, out); break;
    case 13: k_elem<13><<<grid, 256, 0, s>>>(n, x, y, out); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
