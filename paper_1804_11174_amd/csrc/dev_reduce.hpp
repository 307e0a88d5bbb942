// Fixed-order column sums shared by the one-set launchers and the batched
// engine, so that both produce bitwise identical results.
//
// For in[rows][cols]: level 1 sums each block of 256 consecutive rows,
// rows ascending, into L1[b][c]; level 2 sums the level-1 rows, b
// ascending, and applies a scale: out[c] = scale * sum_b L1[b][c].
#pragma once

#include "kde_internal.hpp"

namespace kde {

constexpr int kSumRows = 256;

__device__ __forceinline__ double colsum_level1(const double* __restrict__ in, int64_t rows, int cols, int64_t b,
                                                int c) {
  const int64_t r0 = b * kSumRows;
  const int64_t r1 = min(rows, r0 + kSumRows);
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += in[r * cols + c];
  return s;
}

__device__ __forceinline__ double colsum_level2(const double* __restrict__ l1, int64_t g, int cols, int c,
                                                double scale) {
  double s = 0.0;
  for (int64_t b = 0; b < g; ++b) s += l1[b * cols + c];
  return s * scale;
}

}  // namespace kde
