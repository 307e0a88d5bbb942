// One-set launchers of the particle layout (wrap, pack, stable counting sort
// by angular cell; the device pieces are in dev_layout.hpp) and of the
// fixed-order column sums (dev_reduce.hpp).
//
// The pair sums of the CV objective do not depend on particle order, but a
// wavefront of neighbouring particles lets the pair kernel stop early for
// concentrations at which every pair of the wave is negligible. The sort is
// stable and uses only integer atomics for the histogram counts, so the
// resulting order (and every rounding downstream) is deterministic.
#include "dev_layout.hpp"
#include "dev_reduce.hpp"

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



// Per-block histogram over its contiguous chunk; hist is cell-major
// [cells][blocks] so that one exclusive scan yields stable scatter bases.
template <typename T>
__global__ void __launch_bounds__(kBlock) sort_hist_kernel(const T* __restrict__ x, int64_t n, double L,
                                                          int cells, int64_t chunk,
                                                          int32_t* __restrict__ hist, uint32_t* status) {
  extern __shared__ int32_t lh[];
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  sort_hist_block<T>(x, lo, min(n, lo + chunk), L, cells, blockIdx.x, gridDim.x, lh, hist, status);
}

__global__ void __launch_bounds__(kBlock) exclusive_scan_kernel(int32_t* __restrict__ a, int64_t len) {
  __shared__ int tot[kBlock / 64];
  block_scan_global(a, len, tot);
}

// Stable scatter: the block walks its chunk in rounds of 256 particles; a
// particle's rank among equal cells comes from the lanes before it in its
// wave plus the counts already placed by earlier waves and rounds.
template <typename T, typename P>
__global__ void __launch_bounds__(kBlock) sort_scatter_kernel(const T* __restrict__ x, int64_t n, double L,
                                                             int cells, int64_t chunk,
                                                             const int32_t* __restrict__ base_in,
                                                             P* __restrict__ packed,
                                                             int32_t* __restrict__ perm) {
  extern __shared__ int32_t base[];
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  sort_scatter_block<T, P>(x, lo, min(n, lo + chunk), L, cells, blockIdx.x, gridDim.x, base_in, base, packed, perm);
}

template <typename T, typename P>
kde_status launch_pack_sorted_as(const T* x, int64_t n, double L, const SortPlan& plan, int32_t* hist, P* packed,
                                 int32_t* perm, hipStream_t s, uint32_t* status) {
  const size_t lds = size_t(plan.cells) * sizeof(int32_t);
  hipLaunchKernelGGL(sort_hist_kernel<T>, dim3(plan.blocks), dim3(kBlock), lds, s, x, n, L,
                     plan.cells, plan.chunk, hist, status);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(kBlock), 0, s, hist,
                     int64_t(plan.cells) * plan.blocks);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL((sort_scatter_kernel<T, P>), dim3(plan.blocks), dim3(kBlock), lds, s, x, n, L,
                     plan.cells, plan.chunk, hist, packed, perm);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

template kde_status launch_pack_sorted_as<double, double>(const double*, int64_t, double, const SortPlan&, int32_t*,
                                                          double*, int32_t*, hipStream_t, uint32_t*);
template kde_status launch_pack_sorted_as<float, uint32_t>(const float*, int64_t, double, const SortPlan&, int32_t*,
                                                           uint32_t*, int32_t*, hipStream_t, uint32_t*);
template kde_status launch_pack_sorted_as<double, FracPos>(const double*, int64_t, double, const SortPlan&, int32_t*,
                                                           FracPos*, int32_t*, hipStream_t, uint32_t*);

// ------------------------------------------------------ deterministic sums

// Block (row block x, column block y): one column per thread, kSumCols
// columns per workgroup, so a wide sum spreads its reads over
// ceil(cols / kSumCols) workgroups per row block.
constexpr int kSumCols = 64;

__global__ void __launch_bounds__(kSumCols) colsum_level1_kernel(const double* __restrict__ in, int64_t rows,
                                                                int cols, double* __restrict__ l1) {
  const int c = int(blockIdx.y) * kSumCols + threadIdx.x;
  if (c < cols) l1[int64_t(blockIdx.x) * cols + c] = colsum_level1(in, rows, cols, blockIdx.x, c);
}

__global__ void __launch_bounds__(kSumCols) colsum_level2_kernel(const double* __restrict__ l1, int64_t g, int cols,
                                                                double scale, double* __restrict__ out) {
  const int c = int(blockIdx.x) * kSumCols + threadIdx.x;
  if (c < cols) out[c] = colsum_level2(l1, g, cols, c, scale);
}

// Both levels at once when there is one row block: level 2 over a single
// level-1 row is 0 + l1, exactly l1, so out[c] = l1 * scale has the
// two-kernel result's bits.
__global__ void __launch_bounds__(kSumCols) colsum_single_kernel(const double* __restrict__ in, int64_t rows,
                                                                int cols, double scale, double* __restrict__ out) {
  const int c = int(blockIdx.x) * kSumCols + threadIdx.x;
  if (c < cols) out[c] = colsum_level1(in, rows, cols, 0, c) * scale;
}

size_t column_sum_scratch(int64_t rows, int cols) {
  return size_t(ceil_div(rows, kSumRows)) * size_t(cols) * sizeof(double);
}

kde_status launch_column_sum(const double* in, int64_t rows, int cols, double* scratch, double* out, hipStream_t s,
                             double scale) {
  const int64_t g = ceil_div(rows, kSumRows);
  const unsigned cb = unsigned(ceil_div(cols, kSumCols));
  if (g == 1) {
    hipLaunchKernelGGL(colsum_single_kernel, dim3(cb), dim3(kSumCols), 0, s, in, rows, cols, scale, out);
    KDE_CHECK_LAUNCH();
    return KDE_OK;
  }
  hipLaunchKernelGGL(colsum_level1_kernel, dim3(unsigned(g), cb), dim3(kSumCols), 0, s, in, rows, cols, scratch);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(colsum_level2_kernel, dim3(cb), dim3(kSumCols), 0, s, (const double*)scratch, g, cols, scale,
                     out);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

}  // namespace kde
