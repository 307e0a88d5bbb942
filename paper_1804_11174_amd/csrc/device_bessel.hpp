// Scaled modified Bessel function I0e(x) = exp(-x) I0(x), the normaliser
// of the von Mises kernel (Sec. II.A, Eq. vonMises) and the per-pair factor
// of its two-fold convolution.
//
// Two regimes (coefficients from gen_bessel_coeffs.py):
//   x <  X0: I0(x) = Q(t), t = (x/X0)^2 in [0, 1], a fitted polynomial;
//   x >= X0: sqrt(x) I0e(x) = P(v), v = X0 / x in [0, 1], a fitted polynomial.
// The pieces are exposed separately so that the pair kernels can share the
// per-pair factors 1/x and 1/sqrt(x) across concentrations.
#pragma once

#include <hip/hip_runtime.h>

#include "bessel_coeffs.inc"
#include "exp_table.inc"

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

// I0(x) for x < X0, given t = (x/X0)^2 in [0, 1].
__device__ __forceinline__ double i0_small_f64(double t) {
  constexpr double c[KDE_I0E_F64_NSMALL] = KDE_I0E_F64_SMALL;
  double r = c[KDE_I0E_F64_NSMALL - 1];
#pragma unroll
  for (int k = KDE_I0E_F64_NSMALL - 2; k >= 0; --k) r = fma3(r, t, c[k]);
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
  if (x < KDE_I0E_F64_X0) {
    const double u = x * (1.0 / KDE_I0E_F64_X0);
    return exp(-x) * i0_small_f64(u * u);
  }
  return i0e_sqrt_large_f64(KDE_I0E_F64_X0 / x) / sqrt(x);
}

// ----------------------------------------------------------------- float

// I0(x) for x < X0, given t = (x/X0)^2 in [0, 1].
__device__ __forceinline__ float i0_small_f32(float t) {
  constexpr float c[KDE_I0E_F32_NSMALL] = KDE_I0E_F32_SMALL;
  float r = c[KDE_I0E_F32_NSMALL - 1];
#pragma unroll
  for (int k = KDE_I0E_F32_NSMALL - 2; k >= 0; --k) r = fmaf(r, t, c[k]);
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

// exp(x) for -2^44 <= x <= 0 (or NaN) by Tang's table method: with
// n = rint(x 256/ln2) = 256 m + k, r = x - n ln2/256 (head and tail of
// ln2/256, |r| <= ln2/512), exp(x) = 2^m T[k] (1 + q), T[k] = 2^(k/256) from
// `tab` (KDE_EXP_TABLE, 256 correctly rounded values, staged in LDS by the
// caller) and q = r (1 + r (1/2 + r (1/6 + r/24))) (remainder below 3.8e-17
// relative); T + T q is one FMA. Error below 2 units in the last place.
// The exponent handed to ldexp is limited to -2000 (n >= -512000), so the
// int conversion never overflows and results below ~e^-745 are 0.
__device__ __forceinline__ double exp_nonpos_table(double x, const double* __restrict__ tab) {
  const double n = __builtin_rint(x * KDE_EXP_INV_LN2_256);
  double r = fma(-n, KDE_EXP_LN2_256_HI, x);
  r = fma(-n, KDE_EXP_LN2_256_LO, r);
  const int ni = int(fmax(n, -512000.0));
  const double c24 = 1.0 / 24.0;
  double q = fma3(r, c24, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q *= r;
  const double t = tab[ni & 255];
  return __builtin_amdgcn_ldexp(fma(t, q, t), ni >> 8);
}

// exp(x) for any x <= 0 (or NaN) by the table method, arguments below
// -1000 (far below the underflow limit) clamped first.
__device__ __forceinline__ double exp_nonpos_table_any(double x, const double* __restrict__ tab) {
  return exp_nonpos_table((x < -1000.0) ? -1000.0 : x, tab);  // NaN passes through
}

// exp(x) for any x <= 0 (or NaN): arguments below -1000, far below the
// underflow limit, are clamped first; then as exp_nonpos_f64_bounded.
__device__ __forceinline__ double exp_nonpos_f64(double x) {
  return exp_nonpos_f64_bounded((x < -1000.0) ? -1000.0 : x);  // NaN passes through
}

}  // namespace kde
