// fastmath.hpp -- reciprocal, square root and log2/exp2 for the sweep kernels
// on gfx950, built on the hardware approximations (v_rcp, v_rsq, v_log,
// v_exp) instead of the libm-style sequences.
//
// FP64: v_rcp_f64 / v_rsq_f64 (relative error below 2^-24) followed by one
//   third-order correction: with e the residual of the hardware estimate,
//   1/x = r (1 + e + e^2 + ...) and 1/sqrt(x) = r (1 + e/2 + 3e^2/8 + ...),
//   truncated after e^2, which leaves a truncation error below 2^-72 and the
//   rounding of the last operations (about one ulp) for the positive normal
//   arguments the sweep passes (densities and pressures are floored far above
//   the denormal range).  sqrt(x) = x * (1/sqrt(x)).  log2/exp2 are short
//   polynomials accurate to ~1e-14; root_inv gives x^(-1/k) from an FP32
//   seed and one Newton step.  They only feed the two-rarefaction starting
//   guess, which Newton corrects.
// FP32: the single hardware instructions (about one ulp).
#pragma once
#include <hip/hip_runtime.h>

namespace hydro {
namespace fm {

// ---------------------------------------------------------------- reciprocal
__device__ __forceinline__ double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);  // 1 - x r
  return fma(r, fma(e, e, e), r);    // r (1 + e + e^2)
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------- 1/sqrt
__device__ __forceinline__ double rsqrt(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-x, r * r, 1.0);                // 1 - x r^2
  return fma(r * e, fma(e, 0.375, 0.5), r);            // r (1 + e/2 + 3e^2/8)
}
__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// ---------------------------------------------------------------- sqrt
__device__ __forceinline__ double sqrt(double x) { return x * rsqrt(x); }
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

// x^(-1/k) for a small positive integer k (uniform across the wave) and
// positive x, inv_k = 1/k: an FP32 seed 2^(-log2(x)/k) from the hardware
// log2/exp2 (relative error ~1e-7), then one Newton step on x y^k = 1,
// y <- y (1 - (x y^k - 1)/k), which squares the error (~k 1e-14).  x outside
// the FP32 normal range takes the FP64 polynomial path.
__device__ __forceinline__ double root_inv(double x, int k, double inv_k) {
  if (!(x > 0x1p-120 && x < 0x1p120)) return exp2(-inv_k * log2(x));
  const float lx = __builtin_amdgcn_logf((float)x);
  const double y0 = (double)__builtin_amdgcn_exp2f(-lx * (float)inv_k);
  const double t = fma(x, ipow(y0, k), -1.0);
  return fma(-y0 * inv_k, t, y0);
}
__device__ __forceinline__ float root_inv(float x, int k, float inv_k) {
  (void)k;
  return exp2(-inv_k * log2(x));
}

}  // namespace fm
}  // namespace hydro
