// Kernels of the electrostatic PIC step around the KDE (Sec. III.A) and of
// the uniformity test that drives the width update (Sec. II.D).
//
//  * Poisson and field: net charge rho_q = 1 - L rho (electrons of mean
//    density 1 on a uniform ion background, plasma frequency 1), the
//    three-point periodic Poisson equation phi_{j-1} - 2 phi_j + phi_{j+1}
//    = -dx^2 (rho_q,j - mean rho_q) (the mean carries no field), and the
//    centred field E_j = (phi_{j-1} - phi_{j+1}) / (2 dx). Solved exactly
//    without phi: the half-node fields e_j = (phi_j - phi_{j+1}) / dx obey
//    e_j - e_{j-1} = dx (rho_q,j - mean) and sum to zero over the period,
//    so they are the running sums of that right side less their mean, and
//    E_j = (e_{j-1} + e_j) / 2. One workgroup, three fixed-order block
//    scans in LDS; M a power of two (the session's grids).
//  * Push: v <- v - E_i dt, x <- x + v dt, wrapped into [0, L) (electrons,
//    q/m = -1), one thread per particle.
//  * Field energy: W = (dx / 2) sum_g E_g^2 (eps0 = 1), one workgroup, the
//    squares summed per thread in node order, then across the workgroup in
//    a fixed order; written to one slot of a history (Sec. III.B reads the
//    damping rate off log W).
//  * Anderson-Darling statistic of u = x / L against the uniform law:
//    A^2 = -N - (1/N) sum_j [(2j - 1) ln u_(j) + (2N - 2j + 1) ln(1 - u_(j))]
//    over the sorted u (the usual form with the second logarithm's index
//    reversed), u clamped to [2^-53, 1 - 2^-53]. The positions are sorted by
//    an LSD radix sort, 8 bits per pass, each pass a stable counting sort,
//    on a 32-bit key that orders like the value: the bit pattern in float
//    (non-negative floats order like their unsigned bit patterns), and
//    floor(x 2^32 / L) in double, after which the rare runs of equal keys
//    (positions within L 2^-32 of each other) are put in order by value, so
//    the result is the fully sorted array in four passes instead of eight.
//    Within a pass a wave ranks its lanes by digit from eight ballots and
//    the waves write side by side at offsets from their digit counts. The
//    terms are summed in double in a fixed order.
#include "dev_reduce.hpp"
#include "kde_internal.hpp"

namespace kde {

constexpr int kMaxPoissonM = 2048;  // largest session grid

// Exclusive prefix of x over the kBlock threads of a workgroup in a fixed
// order (a shuffle tree within each wave, then the wave totals in wave
// order); *total gets the workgroup's sum. Every thread calls it; wsum is
// this call's own.
__device__ __forceinline__ double block_exclusive_scan_f64(double x, double* wsum, double* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double v = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  double ex = __shfl_up(v, 1, 64);
  if (lane == 0) ex = 0.0;
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  double pre = 0.0, all = 0.0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w == wave) pre = all;
    all += wsum[w];
  }
  *total = all;
  return pre + ex;
}

__global__ void __launch_bounds__(kBlock) poisson_field_kernel(const double* __restrict__ rho, int M, double L,
                                                              double* __restrict__ E) {
  __shared__ double e[kMaxPoissonM];
  __shared__ double w1[kBlock / 64], w2[kBlock / 64], w3[kBlock / 64];
  const double dx = L / M;
  const int seg = (M + kBlock - 1) / kBlock;
  const int lo = min(M, int(threadIdx.x) * seg), hi = min(M, lo + seg);
  double s = 0.0;  // this thread's cells of the net charge
  for (int j = lo; j < hi; ++j) {
    const double r = 1.0 - L * rho[j];
    e[j] = r;
    s += r;
  }
  double tot;
  block_exclusive_scan_f64(s, w1, &tot);
  const double mean = tot / M;
  double t = 0.0;  // right side dx (rho_q - mean)
  for (int j = lo; j < hi; ++j) {
    const double q = dx * (e[j] - mean);
    e[j] = q;
    t += q;
  }
  double run = block_exclusive_scan_f64(t, w2, &tot);
  double u = 0.0;  // running sums: e_j up to the constant
  for (int j = lo; j < hi; ++j) {
    run += e[j];
    e[j] = run;
    u += run;
  }
  block_exclusive_scan_f64(u, w3, &tot);  // its barrier also publishes e[]
  const double c = -tot / M;
  for (int g = threadIdx.x; g < M; g += kBlock) {
    const int gm = (g == 0) ? M - 1 : g - 1;
    E[g] = 0.5 * ((e[gm] + c) + (e[g] + c));
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) push_kernel(T* __restrict__ x, T* __restrict__ v,
                                                     const T* __restrict__ E_i, int64_t n, double dt, double L) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const T vn = v[i] - E_i[i] * T(dt);
  const double xn = double(x[i] + vn * T(dt));
  double w = xn - L * floor(xn / L);
  if (w >= L) w = 0.0;
  v[i] = vn;
  x[i] = T(w);
}

// ---------------------------------------------------------- radix sort (AD)

// 32-bit sort key, ordered like the value: float bit pattern (positions are
// non-negative), or floor(x kscale) with kscale = 2^32 / L in double (a
// monotone map; ties are ordered afterwards by radix_fixup_kernel).
__device__ __forceinline__ uint32_t sort_key(float v, double) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t sort_key(double v, double kscale) {
  const double q = floor(v * kscale);
  if (!(q > 0.0)) return 0u;  // also NaN
  return q >= 4294967295.0 ? 4294967295u : uint32_t(q);
}

template <typename T>
__device__ __forceinline__ int digit_of(T v, int pass, double kscale) {
  return int((sort_key(v, kscale) >> (8 * pass)) & 0xffu);
}

constexpr int kSortPasses = 4;

template <typename T>
__global__ void __launch_bounds__(kBlock) radix_hist_kernel(const T* __restrict__ in, int64_t n, int64_t chunk, int pass,
                                                           double kscale, int32_t* __restrict__ hist) {
  __shared__ int32_t lh[256];
  lh[threadIdx.x] = 0;
  __syncthreads();
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) atomicAdd(&lh[digit_of(in[i], pass, kscale)], 1);
  __syncthreads();
  hist[int64_t(threadIdx.x) * gridDim.x + blockIdx.x] = lh[threadIdx.x];
}

// Exclusive prefix of x over the kBlock threads of a workgroup (shuffles
// within a wave, then the wave totals through wsum); every thread calls it.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t x, int32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t v = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  int32_t pre = v - x;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  return pre;
}

// One workgroup per digit: exclusive scan, in place, of that digit's row of
// the [digit][block] histogram (the offsets of each block within the digit),
// and the digit's total count into totals[digit].
__global__ void __launch_bounds__(kBlock) radix_scan_kernel(int32_t* __restrict__ hist, int64_t blocks,
                                                            int32_t* __restrict__ totals) {
  __shared__ int32_t wsum[kBlock / 64];
  int32_t* row = hist + int64_t(blockIdx.x) * blocks;
  const int64_t seg = (blocks + kBlock - 1) / kBlock;
  const int64_t lo = int64_t(threadIdx.x) * seg;
  const int64_t hi = min(blocks, lo + seg);
  int32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += row[i];
  int32_t run = block_exclusive_scan(s, wsum);
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t x = row[i];
    row[i] = run;
    run += x;
  }
  if (threadIdx.x == kBlock - 1) totals[blockIdx.x] = run;
}

// Stable scatter of one pass. Per round of kBlock keys: a lane's peers (the
// lanes of its wave with the same digit) come from eight ballots, its rank
// is the number of peers before it; each wave's digit counts go to LDS, and
// every key lands at base[digit] + (the counts of that digit in the waves
// before its own) + rank, so the waves write side by side and the order
// stays that of the input within each digit. base starts as the block's
// offset within its digit plus the totals of the smaller digits.
template <typename T>
__global__ void __launch_bounds__(kBlock) radix_scatter_kernel(const T* __restrict__ in, int64_t n, int64_t chunk,
                                                              int pass, double kscale,
                                                              const int32_t* __restrict__ base_in,
                                                              const int32_t* __restrict__ totals,
                                                              T* __restrict__ out) {
  constexpr int kWaves = kBlock / 64;
  __shared__ int32_t base[256];
  __shared__ int32_t cnt[kWaves][256];
  __shared__ int32_t wsum[kWaves];
  const int tid = threadIdx.x;
  const int32_t below = block_exclusive_scan(totals[tid], wsum);
  base[tid] = base_in[int64_t(tid) * gridDim.x + blockIdx.x] + below;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) cnt[w][tid] = 0;
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes below this one
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int64_t r0 = lo; r0 < hi; r0 += kBlock) {
    const int64_t i = r0 + tid;
    const bool valid = i < hi;
    const T v = valid ? in[i] : T(0);
    const int d = valid ? digit_of(v, pass, kscale) : 0;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) cnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int off = base[d] + rank;
      for (int w = 0; w < wave; ++w) off += cnt[w][d];
      out[off] = v;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      add += cnt[w][tid];
      cnt[w][tid] = 0;
    }
    base[tid] += add;
    __syncthreads();
  }
}

// Double keys map positions within L 2^-32 to one key; after the passes,
// the first thread of every run of equal keys puts its run in order by value
// (insertion sort; runs are disjoint, and a neighbour's key does not change
// while its run is being sorted, so the run boundaries read are stable).
__global__ void __launch_bounds__(kBlock) radix_fixup_kernel(double* __restrict__ a, int64_t n, double kscale) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = sort_key(a[i], kscale);
  if (i > 0 && sort_key(a[i - 1], kscale) == k) return;
  int64_t j = i + 1;
  while (j < n && sort_key(a[j], kscale) == k) ++j;
  for (int64_t p = i + 1; p < j; ++p) {
    const double v = a[p];
    int64_t q = p - 1;
    while (q >= i && a[q] > v) {
      a[q + 1] = a[q];
      --q;
    }
    a[q + 1] = v;
  }
}

// Block b: the A^2 terms of sorted ranks [256 b, 256 b + 256), summed in a
// fixed order into partials[b].
template <typename T>
__global__ void __launch_bounds__(kBlock) ad_terms_kernel(const T* __restrict__ sorted, int64_t n, double L,
                                                         double* __restrict__ partials) {
  __shared__ double red[kBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  double t = 0.0;
  if (i < n) {
    const double lo = 1.1102230246251565e-16, hi = 1.0 - 1.1102230246251565e-16;
    double u = double(sorted[i]) / L;
    u = u < lo ? lo : (u > hi ? hi : u);
    const double j = double(i + 1);
    t = (2.0 * j - 1.0) * log(u) + (2.0 * double(n) - 2.0 * j + 1.0) * log1p(-u);
  }
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    partials[blockIdx.x] = s;
  }
}

__global__ void ad_finish_kernel(const double* __restrict__ sum, int64_t n, double* __restrict__ a2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *a2 = -double(n) - sum[0] / double(n);
}

// ------------------------------------------------------------------ host

size_t poisson_max_m() { return kMaxPoissonM; }

// W of the current field into history slot *step (when the slot exists),
// then *step + 1: the slot index lives on the device, so a captured step
// replays with the same arguments every time.
__global__ void __launch_bounds__(kBlock) field_energy_kernel(const double* __restrict__ E, int M, double half_dx,
                                                             double* __restrict__ energy, int64_t history,
                                                             int64_t* __restrict__ step) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int g = threadIdx.x; g < M; g += kBlock) s = fma(E[g], E[g], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    const int64_t st = *step;
    if (st >= 0 && st < history) energy[st] = half_dx * t;
    *step = st + 1;
  }
}

__global__ void set_step_kernel(int64_t* __restrict__ step, int64_t value) {
  if (threadIdx.x == 0) *step = value;
}

kde_status launch_field_energy(const double* E, int M, double L, double* energy, int64_t history, int64_t* step,
                               hipStream_t s) {
  hipLaunchKernelGGL(field_energy_kernel, dim3(1), dim3(kBlock), 0, s, E, M, 0.5 * (L / M), energy, history, step);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status launch_set_step(int64_t* step, int64_t value, hipStream_t s) {
  hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, s, step, value);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status launch_poisson_field(const double* rho, int M, double L, double* E, hipStream_t s) {
  if (M < 2 || M > kMaxPoissonM || (M & (M - 1))) return fail(KDE_E_INVALID_ARG, "M must be a power of two in [2, %d]", kMaxPoissonM);
  hipLaunchKernelGGL(poisson_field_kernel, dim3(1), dim3(kBlock), 0, s, rho, M, L, E);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

template <typename T>
kde_status launch_push(T* x, T* v, const T* E_i, int64_t n, double dt, double L, hipStream_t s) {
  hipLaunchKernelGGL(push_kernel<T>, dim3(unsigned(ceil_div(n, kBlock))), dim3(kBlock), 0, s, x, v, E_i, n, dt, L);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}
template kde_status launch_push<double>(double*, double*, const double*, int64_t, double, double, hipStream_t);
template kde_status launch_push<float>(float*, float*, const float*, int64_t, double, double, hipStream_t);

static int64_t ad_blocks(int64_t n) {
  int64_t b = ceil_div(n, kBlock);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return b;
}

size_t ad_workspace_bytes(int64_t n, int prec) {
  const int64_t blocks = ad_blocks(n);
  const int64_t tb = ceil_div(n, kBlock);
  Carver c(nullptr, 0);
  c.take<char>(size_t(n) * elem_size(prec));
  c.take<char>(size_t(n) * elem_size(prec));
  c.take<int32_t>(256 * size_t(blocks));
  c.take<int32_t>(256);
  c.take<double>(size_t(tb));
  c.take<double>(column_sum_scratch(tb, 1) / sizeof(double) + 1);
  c.take<double>(1);
  return c.used;
}

// A^2 of positions x[n] (device) into *a2 (device).
template <typename T>
kde_status launch_ad_statistic(const T* x, int64_t n, double L, double* a2, void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t blocks = ad_blocks(n);
  const int64_t chunk = ceil_div(n, blocks);
  const int64_t tb = ceil_div(n, kBlock);
  Carver c(ws, ws_bytes);
  T* buf0 = c.take<T>(size_t(n));
  T* buf1 = c.take<T>(size_t(n));
  int32_t* hist = c.take<int32_t>(256 * size_t(blocks));
  int32_t* totals = c.take<int32_t>(256);
  double* parts = c.take<double>(size_t(tb));
  double* scratch = c.take<double>(column_sum_scratch(tb, 1) / sizeof(double) + 1);
  double* sum = c.take<double>(1);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "AD workspace too small: %zu < %zu", ws_bytes, c.used);
  // The first pass reads x itself; the passes then alternate between the
  // two buffers, the sorted array ending in bufs[(passes - 1) & 1].
  T* bufs[2] = {buf0, buf1};
  const double kscale = 4294967296.0 / L;
  for (int pass = 0; pass < kSortPasses; ++pass) {
    const T* in = pass == 0 ? x : bufs[(pass + 1) & 1];
    T* out = bufs[pass & 1];
    hipLaunchKernelGGL(radix_hist_kernel<T>, dim3(unsigned(blocks)), dim3(kBlock), 0, s, in, n, chunk, pass, kscale,
                       hist);
    KDE_CHECK_LAUNCH();
    hipLaunchKernelGGL(radix_scan_kernel, dim3(256), dim3(kBlock), 0, s, hist, blocks, totals);
    KDE_CHECK_LAUNCH();
    hipLaunchKernelGGL(radix_scatter_kernel<T>, dim3(unsigned(blocks)), dim3(kBlock), 0, s, in, n, chunk, pass, kscale,
                       (const int32_t*)hist, (const int32_t*)totals, out);
    KDE_CHECK_LAUNCH();
  }
  T* src = bufs[(kSortPasses - 1) & 1];
  if constexpr (std::is_same<T, double>::value) {
    hipLaunchKernelGGL(radix_fixup_kernel, dim3(unsigned(ceil_div(n, kBlock))), dim3(kBlock), 0, s, src, n, kscale);
    KDE_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(ad_terms_kernel<T>, dim3(unsigned(tb)), dim3(kBlock), 0, s, (const T*)src, n, L, parts);
  KDE_CHECK_LAUNCH();
  KDE_RETURN_IF(launch_column_sum(parts, tb, 1, scratch, sum, s));
  hipLaunchKernelGGL(ad_finish_kernel, dim3(1), dim3(64), 0, s, (const double*)sum, n, a2);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}
template kde_status launch_ad_statistic<double>(const double*, int64_t, double, double*, void*, size_t, hipStream_t);
template kde_status launch_ad_statistic<float>(const float*, int64_t, double, double*, void*, size_t, hipStream_t);

}  // namespace kde
