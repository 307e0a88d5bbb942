// Device pieces of the particle layout (wrap, pack, stable counting sort by
// angular cell), shared by the one-set kernels of layout.hip and the
// batched engine. A stable sort by cell has one result whatever the block
// decomposition (cell ascending, input index ascending within a cell), so
// both users produce the same packed order.
//
// Packed forms:
//   double: the half-angle vector (cos(pi x / L), sin(pi x / L));
//   float : the phase as a 32-bit fixed-point fraction of the period,
//           u = round(x / L * 2^32) mod 2^32. The difference of two phases
//           in wrapping integer arithmetic is then the exact periodic
//           separation (resolution L / 2^32, far below a float's spacing
//           at L), so close pairs keep full relative accuracy.
#pragma once

#include "kde_internal.hpp"

namespace kde {

// Positions are wrapped in double whatever their storage precision.
__device__ __forceinline__ double wrap_d(double x, double L) {
  double y = x - L * floor(x / L);
  return (y >= L) ? 0.0 : y;
}

template <typename T>
__device__ __forceinline__ int cell_of(T x, double L, int cells) {
  if (!isfinite(double(x))) return 0;  // non-finite: any valid cell, value stays NaN
  const double w = wrap_d(double(x), L);
  int c = int(w * double(cells) / L);
  return c < 0 ? 0 : (c >= cells ? cells - 1 : c);
}

__device__ __forceinline__ void store_packed(double* packed, int64_t dest, double frac) {
  double sp, cp;
  sincospi(frac, &sp, &cp);
  packed[2 * dest] = cp;
  packed[2 * dest + 1] = sp;
}

__device__ __forceinline__ void store_packed(uint32_t* packed, int64_t dest, double frac) {
  // frac in [0, 1): the nearest multiple of 2^-32, wrapped
  const double v = floor(frac * 4294967296.0 + 0.5);
  packed[dest] = (v >= 4294967296.0) ? 0u : uint32_t(v);
}

// Scatter particles [lo, hi) of one block into `packed` in stable cell
// order. `base` (LDS, `cells` ints) holds, per cell, the first destination
// of this block's particles and is advanced as they are placed. The block
// walks its range in rounds of kBlock; a particle's rank among equal cells
// comes from the lanes before it in its wave plus what earlier waves and
// rounds placed. Every thread of the block must call this.
template <typename T, typename P>
__device__ __forceinline__ void stable_scatter(const T* __restrict__ x, int64_t lo, int64_t hi, double L, int cells,
                                               int* base, P* __restrict__ packed, int32_t* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int64_t r0 = lo; r0 < hi; r0 += kBlock) {
    const int64_t i = r0 + threadIdx.x;
    const bool valid = i < hi;
    const T xv = valid ? x[i] : T(0);
    const int c = valid ? cell_of(xv, L, cells) : -1;
    int rank = 0, after = 0;
    for (int k = 0; k < 64; ++k) {
      const int ck = __shfl(c, k, 64);
      if (ck == c) {
        if (k < lane) ++rank;
        if (k > lane) ++after;
      }
    }
    for (int w = 0; w < kBlock / 64; ++w) {
      if (wave == w && valid) {
        const int64_t dest = int64_t(base[c]) + rank;
        store_packed(packed, dest, wrap_d(double(xv), L) / L);
        if (perm) perm[dest] = int32_t(i);
      }
      __syncthreads();
      if (wave == w && valid && after == 0) base[c] += rank + 1;
      __syncthreads();
    }
  }
}

// Exclusive scan of `len` ints held in LDS, by one workgroup: each thread
// scans a contiguous segment, the 256 segment totals are scanned, then each
// segment is offset. `tot` is kBlock ints of LDS scratch.
__device__ __forceinline__ void block_exclusive_scan(int* a, int len, int* tot) {
  const int seg = (len + kBlock - 1) / kBlock;
  const int lo = threadIdx.x * seg;
  const int hi = min(len, lo + seg);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < kBlock; ++t) {
      const int v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int run = tot[threadIdx.x];
  for (int i = lo; i < hi; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
}

// Whole-set stable sort by one workgroup: histogram into `base` (LDS,
// `cells` ints), exclusive scan, then the scatter. `tot` is kBlock ints of
// LDS scratch. Every thread of the block must call this.
template <typename T, typename P>
__device__ __forceinline__ void sort_set_one_block(const T* __restrict__ x, int64_t n, double L, int cells,
                                                   int* base, int* tot, P* __restrict__ packed) {
  for (int c = threadIdx.x; c < cells; c += kBlock) base[c] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += kBlock) atomicAdd(&base[cell_of(x[i], L, cells)], 1);
  __syncthreads();
  block_exclusive_scan(base, cells, tot);
  stable_scatter<T, P>(x, 0, n, L, cells, base, packed, nullptr);
}

}  // namespace kde
