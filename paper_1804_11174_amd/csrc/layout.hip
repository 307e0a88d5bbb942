// Particle layout for the pair kernels: wrap positions into [0, L), pack
// each and order the particles by angular cell with a stable counting sort.
//
// Packed forms:
//   double: the half-angle vector (cos(pi x / L), sin(pi x / L));
//   float : the phase as a 32-bit fixed-point fraction of the period,
//           u = round(x / L * 2^32) mod 2^32. The difference of two phases
//           in wrapping integer arithmetic is then the exact periodic
//           separation (resolution L / 2^32, far below a float's spacing
//           at L), so close pairs keep full relative accuracy.
//
// The pair sums of the CV objective do not depend on particle order, but a
// wavefront of neighbouring particles lets the pair kernel stop early for
// concentrations at which every pair of the wave is negligible. The sort is
// stable and uses only integer atomics for the histogram counts, so the
// resulting order (and every rounding downstream) is deterministic.
#include "kde_internal.hpp"

namespace kde {

SortPlan make_sort_plan(int64_t n) {
  SortPlan p;
  p.n = n;
  int64_t cells = n / 32;
  if (cells < 1) cells = 1;
  if (cells > 8192) cells = 8192;
  p.cells = int(cells);
  int64_t blocks = ceil_div(n, 2048);
  if (blocks < 1) blocks = 1;
  if (blocks > 128) blocks = 128;
  p.blocks = int(blocks);
  p.chunk = ceil_div(n, blocks);
  return p;
}

// Positions are wrapped in double whatever their storage precision.
__device__ __forceinline__ double wrap_d(double x, double L) {
  double y = x - L * floor(x / L);
  return (y >= L) ? 0.0 : y;
}

template <typename T>
__device__ __forceinline__ int cell_of(T x, double L, int cells) {
  if (!isfinite(double(x))) return 0;  // non-finite: any valid cell, value stays NaN
  const double w = wrap_d(double(x), double(L));
  int c = int(w * double(cells) / double(L));
  return c < 0 ? 0 : (c >= cells ? cells - 1 : c);
}

// Per-block histogram over its contiguous chunk; hist is cell-major
// [cells][blocks] so that one exclusive scan yields stable scatter bases.
template <typename T>
__global__ void __launch_bounds__(kBlock) sort_hist_kernel(const T* __restrict__ x, int64_t n, double L,
                                                          int cells, int64_t chunk,
                                                          int32_t* __restrict__ hist) {
  extern __shared__ int32_t lh[];
  for (int c = threadIdx.x; c < cells; c += kBlock) lh[c] = 0;
  __syncthreads();
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) atomicAdd(&lh[cell_of(x[i], L, cells)], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += kBlock) hist[int64_t(c) * gridDim.x + blockIdx.x] = lh[c];
}

// Exclusive scan of `len` ints in place, one workgroup: each thread scans a
// contiguous segment, then the segment totals are scanned in LDS.
__global__ void __launch_bounds__(kBlock) exclusive_scan_kernel(int32_t* __restrict__ a, int64_t len) {
  __shared__ int32_t tot[kBlock];
  const int64_t seg = (len + kBlock - 1) / kBlock;
  const int64_t lo = int64_t(threadIdx.x) * seg;
  const int64_t hi = min(len, lo + seg);
  int32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += a[i];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int t = 0; t < kBlock; ++t) {
      int32_t v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int32_t run = tot[threadIdx.x];
  for (int64_t i = lo; i < hi; ++i) {
    int32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// Stable scatter: the block walks its chunk in rounds of 256 particles; a
// particle's rank among equal cells comes from the lanes before it in its
// wave plus the counts already placed by earlier waves and rounds.
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

template <typename T, typename P>
__global__ void __launch_bounds__(kBlock) sort_scatter_kernel(const T* __restrict__ x, int64_t n, double L,
                                                             int cells, int64_t chunk,
                                                             const int32_t* __restrict__ base_in,
                                                             P* __restrict__ packed,
                                                             int32_t* __restrict__ perm) {
  extern __shared__ int32_t base[];
  for (int c = threadIdx.x; c < cells; c += kBlock) base[c] = base_in[int64_t(c) * gridDim.x + blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int64_t r0 = lo; r0 < hi; r0 += kBlock) {
    const int64_t i = r0 + threadIdx.x;
    const bool valid = i < hi;
    T xv = valid ? x[i] : T(0);
    int c = valid ? cell_of(xv, L, cells) : -1;
    // rank among earlier lanes of this wave with the same cell, and whether
    // this lane is the last of its cell in the wave
    int rank = 0, after = 0;
    for (int k = 0; k < 64; ++k) {
      int ck = __shfl(c, k, 64);
      if (ck == c) {
        if (k < lane) ++rank;
        if (k > lane) ++after;
      }
    }
    for (int w = 0; w < kBlock / 64; ++w) {
      if (wave == w && valid) {
        int dest = base[c] + rank;
        const double wx = wrap_d(double(xv), double(L));
        store_packed(packed, dest, wx / double(L));
        if (perm) perm[dest] = int32_t(i);
      }
      __syncthreads();
      if (wave == w && valid && after == 0) base[c] += rank + 1;
      __syncthreads();
    }
  }
}

template <typename T>
kde_status launch_pack_sorted(const T* x, int64_t n, double L, const SortPlan& plan, int32_t* hist,
                              typename Packed<T>::type* packed, int32_t* perm, hipStream_t s) {
  const size_t lds = size_t(plan.cells) * sizeof(int32_t);
  hipLaunchKernelGGL(sort_hist_kernel<T>, dim3(plan.blocks), dim3(kBlock), lds, s, x, n, L,
                     plan.cells, plan.chunk, hist);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(kBlock), 0, s, hist,
                     int64_t(plan.cells) * plan.blocks);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL((sort_scatter_kernel<T, typename Packed<T>::type>), dim3(plan.blocks), dim3(kBlock), lds, s, x, n, L,
                     plan.cells, plan.chunk, hist, packed, perm);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

template kde_status launch_pack_sorted<double>(const double*, int64_t, double, const SortPlan&,
                                               int32_t*, double*, int32_t*, hipStream_t);
template kde_status launch_pack_sorted<float>(const float*, int64_t, double, const SortPlan&,
                                              int32_t*, uint32_t*, int32_t*, hipStream_t);

// ------------------------------------------------------ deterministic sums

// Stage 1: block b sums rows [b*256, (b+1)*256) for every column; thread
// layout: column = tid mod cols_per_pass, and each thread walks its rows in
// order. Stage 2 (same kernel, one block) sums the stage-1 rows.
__global__ void __launch_bounds__(kBlock) column_sum_kernel(const double* __restrict__ in, int64_t rows,
                                                           int cols, double scale, double* __restrict__ out) {
  const int64_t r0 = int64_t(blockIdx.x) * kBlock;
  const int64_t r1 = min(rows, r0 + kBlock);
  for (int c = threadIdx.x; c < cols; c += kBlock) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += in[r * cols + c];
    out[int64_t(blockIdx.x) * cols + c] = s * scale;
  }
}

size_t column_sum_scratch(int64_t rows, int cols) {
  // ping-pong halves, each large enough for the first stage's output
  return 2 * size_t(ceil_div(rows, kBlock)) * size_t(cols) * sizeof(double) + 512;
}

kde_status launch_column_sum(const double* in, int64_t rows, int cols, double* scratch, double* out,
                             hipStream_t s, double scale) {
  const size_t half = round_up(size_t(ceil_div(rows, kBlock)) * size_t(cols), 32);
  double* buf[2] = {scratch, scratch + half};
  const double* src = in;
  int which = 0;
  while (true) {
    int64_t g = ceil_div(rows, kBlock);
    double* dst = (g <= 1) ? out : buf[which];
    hipLaunchKernelGGL(column_sum_kernel, dim3(unsigned(g < 1 ? 1 : g)), dim3(kBlock), 0, s, src, rows,
                       cols, (g <= 1) ? scale : 1.0, dst);
    KDE_CHECK_LAUNCH();
    if (g <= 1) return KDE_OK;
    src = dst;
    rows = g;
    which ^= 1;
  }
}

}  // namespace kde
