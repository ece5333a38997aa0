// fastmath.hpp -- reciprocal, square root and log2/exp2 for the sweep kernels
// on gfx950, built on the hardware approximations (v_rcp, v_rsq, v_log,
// v_exp) instead of the libm-style sequences.
//
// FP64: v_rcp_f64 / v_rsq_f64 followed by two Newton-Raphson steps (error
//   about one ulp for positive normal arguments, which is all the sweep
//   passes: densities and pressures are floored far above the denormal
//   range).  log2/exp2 are short polynomials accurate to ~1e-14; they only
//   feed the two-rarefaction starting guess, which Newton corrects.
// FP32: the single hardware instructions (about one ulp).
#pragma once
#include <hip/hip_runtime.h>

namespace hydro {
namespace fm {

// ---------------------------------------------------------------- reciprocal
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- 1/sqrt
__device__ __forceinline__ double rsqrt(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  double e = fma(-hx * r, r, 0.5);
  r = fma(r, e, r);
  e = fma(-hx * r, r, 0.5);
  return fma(r, e, r);
}
__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// ---------------------------------------------------------------- sqrt
__device__ __forceinline__ double sqrt(double x) {
  // g = x r, h = r/2 refined together (Goldschmidt form)
  const double r0 = __builtin_amdgcn_rsq(x);
  double g = x * r0;
  double h = 0.5 * r0;
  double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}
__device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------- log2 / exp2
// log2 for positive normal x: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716, series to s^15.
__device__ __forceinline__ double log2(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < 0.70710678118654752440) {
    m = m + m;
    e -= 1;
  }
  const double s = (m - 1.0) * rcp(m + 1.0);
  const double s2 = s * s;
  double p = 1.0 / 15.0;
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  p = fma(p, s2, 1.0);
  const double ln_m = 2.0 * s * p;
  return fma(ln_m, 1.44269504088896340736, (double)e);  // e + ln(m)/ln(2)
}
__device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }

// exp2 for |y| < 1000: 2^n e^(f ln 2), n = rint(y), |f| <= 1/2, Taylor to t^11.
__device__ __forceinline__ double exp2(double y) {
  const double n = rint(y);
  const double t = (y - n) * 0.69314718055994530942;
  double p = 1.0 / 39916800.0;  // 1/11!
  p = fma(p, t, 1.0 / 3628800.0);
  p = fma(p, t, 1.0 / 362880.0);
  p = fma(p, t, 1.0 / 40320.0);
  p = fma(p, t, 1.0 / 5040.0);
  p = fma(p, t, 1.0 / 720.0);
  p = fma(p, t, 1.0 / 120.0);
  p = fma(p, t, 1.0 / 24.0);
  p = fma(p, t, 1.0 / 6.0);
  p = fma(p, t, 0.5);
  p = fma(p, t, 1.0);
  p = fma(p, t, 1.0);
  return __builtin_amdgcn_ldexp(p, (int)n);
}
__device__ __forceinline__ float exp2(float y) { return __builtin_amdgcn_exp2f(y); }

// x^a for positive normal x (starting guesses only)
template <typename T>
__device__ __forceinline__ T pow_pos(T x, T a) {
  return exp2(a * log2(x));
}

// x^k for a small positive integer k (uniform across the wave)
template <typename T>
__device__ __forceinline__ T ipow(T x, int k) {
  T r = T(1);
  T b = x;
  while (k > 0) {
    if (k & 1) r *= b;
    b *= b;
    k >>= 1;
  }
  return r;
}

}  // namespace fm
}  // namespace hydro
