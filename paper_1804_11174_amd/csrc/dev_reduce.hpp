// Fixed-order column sums shared by the one-set launchers and the batched
// engine, so that both produce bitwise identical results.
//
// For in[rows][cols]: level 1 sums each block of 128 consecutive rows,
// rows ascending, into L1[b][c]; level 2 sums the level-1 rows, b
// ascending, and applies a scale: out[c] = scale * sum_b L1[b][c].
#pragma once

#include "kde_internal.hpp"

namespace kde {

constexpr int kSumRows = 128;  // rows per level-1 block: the length of one column's add chain

// Rows are loaded kLoadAhead at a time and then added one by one, in
// ascending order: the same sum as the plain loop, with the loads of a
// batch in flight together instead of one dependent load per add.
constexpr int kLoadAhead = 32;

__device__ __forceinline__ double column_run(const double* __restrict__ in, int64_t r0, int64_t r1, int cols, int c) {
  double s = 0.0;
  int64_t r = r0;
  for (; r + kLoadAhead <= r1; r += kLoadAhead) {
    double v[kLoadAhead];
#pragma unroll
    for (int k = 0; k < kLoadAhead; ++k) v[k] = in[(r + k) * cols + c];
#pragma unroll
    for (int k = 0; k < kLoadAhead; ++k) s += v[k];
  }
  for (; r < r1; ++r) s += in[r * cols + c];
  return s;
}

__device__ __forceinline__ double colsum_level1(const double* __restrict__ in, int64_t rows, int cols, int64_t b,
                                                int c) {
  const int64_t r0 = b * kSumRows;
  return column_run(in, r0, min(rows, r0 + kSumRows), cols, c);
}

__device__ __forceinline__ double colsum_level2(const double* __restrict__ l1, int64_t g, int cols, int c,
                                                double scale) {
  return column_run(l1, 0, g, cols, c) * scale;
}

}  // namespace kde
