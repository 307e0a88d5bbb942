// Scaled modified Bessel function I0e(x) = exp(-x) I0(x), the normaliser
// of the von Mises kernel (Sec. II.A, Eq. vonMises) and the per-pair factor
// of its two-fold convolution.
//
// Two regimes (coefficients from gen_bessel_coeffs.py):
//   x <  X0: I0(x) by its power series in y = x^2, sum_k y^k / (4^k (k!)^2);
//   x >= X0: sqrt(x) I0e(x) = P(u), u = (1/x - C) / H, a fitted polynomial.
// The pieces are exposed separately so that the pair kernels can share the
// per-pair factors 1/x and 1/sqrt(x) across concentrations.
#pragma once

#include <hip/hip_runtime.h>

#include "bessel_coeffs.inc"

namespace kde {

// ---------------------------------------------------------------- double

__host__ __device__ __forceinline__ double i0_series_f64(double y) {
  constexpr double c[KDE_I0E_F64_NSERIES] = KDE_I0E_F64_SERIES;
  double r = c[KDE_I0E_F64_NSERIES - 1];
#pragma unroll
  for (int k = KDE_I0E_F64_NSERIES - 2; k >= 0; --k) r = fma(r, y, c[k]);
  return r;
}

// sqrt(x) * I0e(x) for x >= X0, given t = 1/x.
__host__ __device__ __forceinline__ double i0e_sqrt_large_f64(double t) {
  constexpr double c[KDE_I0E_F64_NFIT] = KDE_I0E_F64_FIT;
  const double u = (t - KDE_I0E_F64_C) * (1.0 / KDE_I0E_F64_H);
  double r = c[KDE_I0E_F64_NFIT - 1];
#pragma unroll
  for (int k = KDE_I0E_F64_NFIT - 2; k >= 0; --k) r = fma(r, u, c[k]);
  return r;
}

__host__ __device__ __forceinline__ double i0e_f64(double x) {
  x = fabs(x);
  if (x < KDE_I0E_F64_X0) return exp(-x) * i0_series_f64(x * x);
  return i0e_sqrt_large_f64(1.0 / x) / sqrt(x);
}

// ----------------------------------------------------------------- float

__device__ __forceinline__ float i0_series_f32(float y) {
  constexpr float c[KDE_I0E_F32_NSERIES] = KDE_I0E_F32_SERIES;
  float r = c[KDE_I0E_F32_NSERIES - 1];
#pragma unroll
  for (int k = KDE_I0E_F32_NSERIES - 2; k >= 0; --k) r = fmaf(r, y, c[k]);
  return r;
}

__device__ __forceinline__ float i0e_sqrt_large_f32(float t) {
  constexpr float c[KDE_I0E_F32_NFIT] = KDE_I0E_F32_FIT;
  const float u = (t - KDE_I0E_F32_C) * (1.0f / KDE_I0E_F32_H);
  float r = c[KDE_I0E_F32_NFIT - 1];
#pragma unroll
  for (int k = KDE_I0E_F32_NFIT - 2; k >= 0; --k) r = fmaf(r, u, c[k]);
  return r;
}

}  // namespace kde
