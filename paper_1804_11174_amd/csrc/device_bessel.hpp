// Scaled modified Bessel function I0e(x) = exp(-x) I0(x), the normaliser
// of the von Mises kernel (Sec. II.A, Eq. vonMises) and the per-pair factor
// of its two-fold convolution.
//
// Two regimes (coefficients from gen_bessel_coeffs.py):
//   x <  X0: I0(x) by its power series in y = x^2, sum_k y^k / (4^k (k!)^2);
//   x >= X0: sqrt(x) I0e(x) = P(v), v = X0 / x in [0, 1], a fitted polynomial.
// The pieces are exposed separately so that the pair kernels can share the
// per-pair factors 1/x and 1/sqrt(x) across concentrations.
#pragma once

#include <hip/hip_runtime.h>

#include "bessel_coeffs.inc"

namespace kde {

// ---------------------------------------------------------------- double

// a * b + c in double as one three-operand v_fma_f64 whose addend c, a
// polynomial coefficient known at compile time, sits in a scalar register
// pair. Left to itself the compiler keeps every coefficient of the kernel's
// polynomials in vector registers for the whole loop (over 100 of them in
// the pair kernel, which halves its occupancy) and uses the two-address
// v_fmac, which needs a copy of the addend before each use. c must be the
// same in every lane.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
}

__device__ __forceinline__ double i0_series_f64(double y) {
  constexpr double c[KDE_I0E_F64_NSERIES] = KDE_I0E_F64_SERIES;
  double r = c[KDE_I0E_F64_NSERIES - 1];
#pragma unroll
  for (int k = KDE_I0E_F64_NSERIES - 2; k >= 0; --k) r = fma3(r, y, c[k]);
  return r;
}

// sqrt(x) * I0e(x) for x >= X0, given v = X0 / x in [0, 1].
__device__ __forceinline__ double i0e_sqrt_large_f64(double v) {
  constexpr double c[KDE_I0E_F64_NFIT] = KDE_I0E_F64_FIT;
  double r = c[KDE_I0E_F64_NFIT - 1];
#pragma unroll
  for (int k = KDE_I0E_F64_NFIT - 2; k >= 0; --k) r = fma3(r, v, c[k]);
  return r;
}

__device__ __forceinline__ double i0e_f64(double x) {
  x = fabs(x);
  if (x < KDE_I0E_F64_X0) return exp(-x) * i0_series_f64(x * x);
  return i0e_sqrt_large_f64(KDE_I0E_F64_X0 / x) / sqrt(x);
}

// ----------------------------------------------------------------- float

__device__ __forceinline__ float i0_series_f32(float y) {
  constexpr float c[KDE_I0E_F32_NSERIES] = KDE_I0E_F32_SERIES;
  float r = c[KDE_I0E_F32_NSERIES - 1];
#pragma unroll
  for (int k = KDE_I0E_F32_NSERIES - 2; k >= 0; --k) r = fmaf(r, y, c[k]);
  return r;
}

// sqrt(x) * I0e(x) for x >= X0, given v = X0 / x in [0, 1].
__device__ __forceinline__ float i0e_sqrt_large_f32(float v) {
  constexpr float c[KDE_I0E_F32_NFIT] = KDE_I0E_F32_FIT;
  float r = c[KDE_I0E_F32_NFIT - 1];
#pragma unroll
  for (int k = KDE_I0E_F32_NFIT - 2; k >= 0; --k) r = fmaf(r, v, c[k]);
  return r;
}

// exp(x) for -2^40 <= x <= 0 in double: x = n ln2 + r with |r| <= ln2/2
// (two-part ln2, Cody and Waite), e^r by its Taylor series to degree 13
// (remainder below 5e-18 relative), then scaled by 2^n. Arguments below
// about -745 give 0 through the scaling (the exponent handed to ldexp is
// limited to -2000, so its conversion to int never overflows; r stays in
// the polynomial's range while x log2(e) keeps its units digit, which
// |x| <= 2^40 leaves room for); NaN gives NaN.
__device__ __forceinline__ double exp_nonpos_f64_bounded(double x) {
  const double n = __builtin_rint(x * 1.4426950408889634);
  double r = fma(-n, 0.6931471805599453094, x);
  r = fma(-n, 2.3190468138462996e-17, r);
  double p = 1.0 / 6227020800.0;
  p = fma3(p, r, 1.0 / 479001600.0);
  p = fma3(p, r, 1.0 / 39916800.0);
  p = fma3(p, r, 1.0 / 3628800.0);
  p = fma3(p, r, 1.0 / 362880.0);
  p = fma3(p, r, 1.0 / 40320.0);
  p = fma3(p, r, 1.0 / 5040.0);
  p = fma3(p, r, 1.0 / 720.0);
  p = fma3(p, r, 1.0 / 120.0);
  p = fma3(p, r, 1.0 / 24.0);
  p = fma3(p, r, 1.0 / 6.0);
  p = fma3(p, r, 0.5);
  p = fma3(p, r, 1.0);
  p = fma3(p, r, 1.0);
  return __builtin_amdgcn_ldexp(p, int(fmax(n, -2000.0)));
}

// exp(x) for any x <= 0 (or NaN): arguments below -1000, far below the
// underflow limit, are clamped first; then as exp_nonpos_f64_bounded.
__device__ __forceinline__ double exp_nonpos_f64(double x) {
  return exp_nonpos_f64_bounded((x < -1000.0) ? -1000.0 : x);  // NaN passes through
}

}  // namespace kde
