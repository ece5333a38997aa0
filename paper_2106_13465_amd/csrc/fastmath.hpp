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
//   the denormal range).  Measured on MI355X over 4M arguments spread over
//   2^-20..2^20: the hardware estimates are good to 2^-24.4 (rcp) and 2^-24.2
//   (rsq); after the correction 1.1e-16 and 1.6e-16, with 99.98% and 87% of
//   the results correctly rounded, where a second-order correction would
//   leave 2.2e-15 and 4.1e-15.  sqrt(x) = x * (1/sqrt(x)).  Fractional powers
//   for starting guesses are range-reduced onto the FP32 instructions;
//   x^(-1/k) adds one FP64 Newton step (two where the power enters the
//   result: the exact solver's wave curves).
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
// FP32 hardware instructions.  The FP64 kernels take fractional powers only
// for the two-rarefaction starting guess, which Newton corrects, through the
// range-reduced forms below, so no FP64 polynomial (and none of its constants
// held in registers) sits in the sweeps.
__device__ __forceinline__ float log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float exp2(float y) { return __builtin_amdgcn_exp2f(y); }

// x^k for a small positive integer k (uniform across the wave).  The
// exponents of the usual ratios of specific heats (3, 5, 7: gamma = 5/3, 7/5)
// take a fixed chain of multiplications behind a scalar branch on k; any other
// k the binary method, whose loop and selects cost three times as many vector
// instructions.  Both multiply the same factors in the same order (x x^2 x^4
// for k = 7), so the result does not depend on the path.
template <typename T>
__device__ __forceinline__ T ipow(T x, int k) {
  if (k == 7) {
    const T x2 = x * x;
    return (x * x2) * (x2 * x2);
  }
  if (k == 5) {
    const T x2 = x * x;
    return x * (x2 * x2);
  }
  if (k == 3) return x * (x * x);
  T r = T(1);
  T b = x;
  while (k > 0) {
    if (k & 1) r *= b;
    b *= b;
    k >>= 1;
  }
  return r;
}

// x^a for positive normal x (starting guesses only).  FP64: x = m 2^e with
// m in [1/2, 1), a log2 x = a e + a log2 m = n + f with n an integer and
// |f| <= 1/2, result 2^f 2^n with 2^f and log2 m from the FP32 instructions
// (relative error ~1e-7, for any exponent the double range holds).
__device__ __forceinline__ double pow_pos(double x, double a) {
  const double e = (double)__builtin_amdgcn_frexp_exp(x);
  const float lm = __builtin_amdgcn_logf((float)__builtin_amdgcn_frexp_mant(x));
  const double t = a * (e + (double)lm);
  const double n = rint(t);
  return __builtin_amdgcn_ldexp((double)__builtin_amdgcn_exp2f((float)(t - n)), (int)n);
}
__device__ __forceinline__ float pow_pos(float x, float a) { return exp2(a * log2(x)); }

// x^(-1/k) for a small positive integer k (uniform across the wave) and
// positive normal x, inv_k = 1/k.  FP64: x = x' 2^(k m) with m = rint(e/k)
// for x's binary exponent e, so x' lies within a factor 2^(k/2 + 1) of 1; an
// FP32 seed y' = 2^(-log2(x')/k) (relative error ~1e-7), one Newton step on
// x' y^k = 1, y' <- y' (1 - (x' y'^k - 1)/k), which squares the error
// (~k 1e-14), and the result y' 2^(-m).
__device__ __forceinline__ double root_inv(double x, int k, double inv_k) {
  const int m = (int)rint((double)__builtin_amdgcn_frexp_exp(x) * inv_k);
  const double xr = __builtin_amdgcn_ldexp(x, -k * m);
  const float lx = __builtin_amdgcn_logf((float)xr);
  const double y0 = (double)__builtin_amdgcn_exp2f(-lx * (float)inv_k);
  const double t = fma(xr, ipow(y0, k), -1.0);
  return __builtin_amdgcn_ldexp(fma(-y0 * inv_k, t, y0), -m);
}
__device__ __forceinline__ float root_inv(float x, int k, float inv_k) {
  (void)k;
  return exp2(-inv_k * log2(x));
}

// (a/b)^(-1/k) for positive normal a, b within the FP32 range (pressures:
// floored, finite) and x = a/b computed by the caller in FP64: an FP32 seed
// 2^(-(log2 a - log2 b)/k) from the two FP32 logarithms (no range reduction
// needed: a and b are FP32 numbers even where their ratio is not) and one
// FP64 Newton step on x y^k = 1.  The seed's relative error is about 1e-7
// times max(1, |log2 a|, |log2 b|) / k, and the step squares it (below
// 3e-12 for pressures in 1e-20..1e20), ample for a starting guess.
__device__ __forceinline__ double root_inv_ratio(double a, double b, double x, int k,
                                                 double inv_k) {
  const float la = __builtin_amdgcn_logf((float)a), lb = __builtin_amdgcn_logf((float)b);
  const double y0 = (double)__builtin_amdgcn_exp2f((lb - la) * (float)inv_k);
  const double t = fma(x, ipow(y0, k), -1.0);
  return fma(-y0 * inv_k, t, y0);
}
__device__ __forceinline__ float root_inv_ratio(float a, float b, float x, int k, float inv_k) {
  (void)a;
  (void)b;
  return root_inv(x, k, inv_k);
}

// x^(-1/k) to full precision (the exact Riemann solver's wave curves, where
// the power enters the result rather than a starting guess): a second Newton
// step after root_inv takes the ~k 1e-14 error to rounding level.
__device__ __forceinline__ double root_inv_full(double x, int k, double inv_k) {
  const double y = root_inv(x, k, inv_k);
  return fma(-y * inv_k, fma(x, ipow(y, k), -1.0), y);
}
__device__ __forceinline__ float root_inv_full(float x, int k, float inv_k) {
  return root_inv(x, k, inv_k);
}

// x^a for positive normal x to full precision, any exponent: the device
// library's pow in FP64 (only for ratios of specific heats whose exponents
// are not integers), the FP32 instructions in FP32.
__device__ __forceinline__ double pow_full(double x, double a) { return ::pow(x, a); }
__device__ __forceinline__ float pow_full(float x, float a) { return pow_pos(x, a); }

}  // namespace fm
}  // namespace hydro
