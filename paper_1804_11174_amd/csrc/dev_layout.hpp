// Device pieces of the particle layout (wrap, pack, stable counting sort by
// angular cell), shared by the one-set kernels of layout.hip and the
// batched engine. A stable sort by cell has one result whatever the block
// decomposition (cell ascending, input index ascending within a cell), so
// both users produce the same packed order.
//
// Packed forms:
//   double: the half-angle vector (cos(pi w / L), sin(pi w / L)) and the
//           wrapped position w itself (the difference of two close w is
//           exact, which the pair kernel uses for near-coincident pairs);
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

// Store the packed form of a particle at wrapped position w in [0, L).
__device__ __forceinline__ void store_packed(double* packed, int64_t dest, double w, double L) {
  double sp, cp;
  sincospi(w / L, &sp, &cp);
  packed[3 * dest] = cp;
  packed[3 * dest + 1] = sp;
  packed[3 * dest + 2] = w;
}

__device__ __forceinline__ void store_packed(FracPos* packed, int64_t dest, double w, double L) {
  packed[dest].f = w / L;
}

__device__ __forceinline__ void store_packed(uint32_t* packed, int64_t dest, double w, double L) {
  // w / L in [0, 1): the nearest multiple of 2^-32, wrapped
  const double v = floor((w / L) * 4294967296.0 + 0.5);
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
        store_packed(packed, dest, wrap_d(double(xv), L), L);
        if (perm) perm[dest] = int32_t(i);
      }
      __syncthreads();
      if (wave == w && valid && after == 0) base[c] += rank + 1;
      __syncthreads();
    }
  }
}

// Exclusive scan of `len` ints in global memory, in place, by one
// workgroup. The array is walked in tiles of 4 * kBlock: each lane holds
// four consecutive elements, lane totals are scanned across the wave with
// shuffles and the wave totals through LDS, and a running carry joins the
// tiles. `tot` is kBlock / 64 ints of LDS. Every thread must call this.
__device__ __forceinline__ void block_scan_global(int32_t* __restrict__ a, int64_t len, int* tot) {
  constexpr int kWaves = kBlock / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int carry = 0;
  for (int64_t t0 = 0; t0 < len; t0 += 4 * kBlock) {
    const int64_t i0 = t0 + 4 * int64_t(threadIdx.x);
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (i0 + k < len) ? a[i0 + k] : 0;
    const int own = v[0] + v[1] + v[2] + v[3];
    int incl = own;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    if (lane == 63) tot[wave] = incl;
    __syncthreads();
    int woff = 0, tile = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const int tw = tot[w];
      if (w < wave) woff += tw;
      tile += tw;
    }
    int run = carry + woff + incl - own;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < len) a[i0 + k] = run;
      run += v[k];
    }
    carry += tile;
    __syncthreads();  // tot is rewritten by the next tile
  }
}

// Sort block `b` of `nblocks` over particles [lo, hi): its cell histogram,
// counted in LDS `lh` (cells ints) with integer atomics, is stored as
// column b of the cell-major [cells][nblocks] array `hist`, so that one
// exclusive scan of `hist` gives every block its stable scatter bases.
// Non-finite positions are noted in `status` (may be null).
template <typename T>
__device__ __forceinline__ void sort_hist_block(const T* __restrict__ x, int64_t lo, int64_t hi, double L, int cells,
                                                int b, int nblocks, int* lh, int32_t* __restrict__ hist,
                                                uint32_t* status) {
  for (int c = threadIdx.x; c < cells; c += kBlock) lh[c] = 0;
  __syncthreads();
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
    const T xv = x[i];
    note_numeric(status, !isfinite(double(xv)), false);
    atomicAdd(&lh[cell_of(xv, L, cells)], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += kBlock) hist[int64_t(c) * nblocks + b] = lh[c];
}

// Sort block `b`: load its scanned bases from `hist` into LDS `base` and
// scatter particles [lo, hi) stably.
template <typename T, typename P>
__device__ __forceinline__ void sort_scatter_block(const T* __restrict__ x, int64_t lo, int64_t hi, double L,
                                                   int cells, int b, int nblocks, const int32_t* __restrict__ hist,
                                                   int* base, P* __restrict__ packed, int32_t* __restrict__ perm) {
  for (int c = threadIdx.x; c < cells; c += kBlock) base[c] = hist[int64_t(c) * nblocks + b];
  __syncthreads();
  stable_scatter<T, P>(x, lo, hi, L, cells, base, packed, perm);
}

}  // namespace kde
