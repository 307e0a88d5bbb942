// Kernels of the electrostatic PIC step around the KDE (Sec. III.A) and of
// the uniformity test that drives the width update (Sec. II.D).
//
//  * Poisson and field: net charge rho_q = 1 - L rho (electrons of mean
//    density 1 on a uniform ion background, plasma frequency 1), the
//    three-point periodic Poisson equation solved exactly in Fourier space
//    (mode m is divided by (2 - 2 cos(2 pi m / M)) / dx^2, the mean mode is
//    dropped), then the centred field E_j = (phi_{j-1} - phi_{j+1}) / (2 dx).
//    One workgroup: an iterative radix-2 complex FFT in LDS, M a power of two.
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
//    an LSD radix sort on their bit patterns (non-negative floating-point
//    values order like their unsigned bit patterns), 8 bits per pass, each
//    pass a stable counting sort; the terms are summed in double in a fixed
//    order.
#include "dev_reduce.hpp"
#include "kde_internal.hpp"

namespace kde {

constexpr int kMaxFftM = 2048;

__device__ __forceinline__ int bit_reverse(int v, int bits) { return int(__brev(unsigned(v)) >> (32 - bits)); }

// In-place radix-2 FFT of (re, im)[M] in LDS by one workgroup; sign = -1
// forward, +1 inverse (unscaled).
__device__ void fft_lds(double* re, double* im, int M, int bits, double sign) {
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const int j = bit_reverse(i, bits);
    if (j > i) {
      const double tr = re[i], ti = im[i];
      re[i] = re[j];
      im[i] = im[j];
      re[j] = tr;
      im[j] = ti;
    }
  }
  __syncthreads();
  for (int len = 2; len <= M; len <<= 1) {
    const int half = len >> 1;
    for (int t = threadIdx.x; t < M / 2; t += blockDim.x) {
      const int grp = t / half, k = t % half;
      const int i = grp * len + k, j = i + half;
      double s, c;
      sincospi(sign * 2.0 * double(k) / double(len), &s, &c);
      const double xr = re[j] * c - im[j] * s;
      const double xi = re[j] * s + im[j] * c;
      re[j] = re[i] - xr;
      im[j] = im[i] - xi;
      re[i] += xr;
      im[i] += xi;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) poisson_field_kernel(const double* __restrict__ rho, int M, int bits,
                                                              double L, double* __restrict__ E,
                                                              double* __restrict__ phi_out) {
  __shared__ double re[kMaxFftM], im[kMaxFftM];
  const double dx = L / M;
  for (int g = threadIdx.x; g < M; g += kBlock) {
    re[g] = 1.0 - L * rho[g];
    im[g] = 0.0;
  }
  __syncthreads();
  fft_lds(re, im, M, bits, -1.0);
  for (int m = threadIdx.x; m < M; m += kBlock) {
    if (m == 0) {
      re[0] = 0.0;
      im[0] = 0.0;
    } else {
      const double sp = sinpi(double(m) / double(M));   // 2 - 2 cos(2 pi m / M) = 4 sin^2(pi m / M)
      const double f = dx * dx / (4.0 * sp * sp) / double(M);
      re[m] *= f;
      im[m] *= f;
    }
  }
  __syncthreads();
  fft_lds(re, im, M, bits, 1.0);
  for (int g = threadIdx.x; g < M; g += kBlock) {
    const int gm = (g == 0) ? M - 1 : g - 1;
    const int gp = (g + 1 == M) ? 0 : g + 1;
    E[g] = (re[gm] - re[gp]) / (2.0 * dx);
    if (phi_out) phi_out[g] = re[g];
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

template <typename T>
struct KeyOf;
template <>
struct KeyOf<double> {
  using K = unsigned long long;
  static __device__ __forceinline__ K key(double v) { return K(__double_as_longlong(v)); }
  static constexpr int passes = 8;
};
template <>
struct KeyOf<float> {
  using K = unsigned int;
  static __device__ __forceinline__ K key(float v) { return K(__float_as_uint(v)); }
  static constexpr int passes = 4;
};

template <typename T>
__device__ __forceinline__ int digit_of(T v, int pass) {
  return int((KeyOf<T>::key(v) >> (8 * pass)) & 0xff);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) radix_hist_kernel(const T* __restrict__ in, int64_t n, int64_t chunk, int pass,
                                                           int32_t* __restrict__ hist) {
  __shared__ int32_t lh[256];
  lh[threadIdx.x] = 0;
  __syncthreads();
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) atomicAdd(&lh[digit_of(in[i], pass)], 1);
  __syncthreads();
  hist[int64_t(threadIdx.x) * gridDim.x + blockIdx.x] = lh[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) radix_scan_kernel(int32_t* __restrict__ a, int64_t len) {
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
      const int32_t v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int32_t run = tot[threadIdx.x];
  for (int64_t i = lo; i < hi; ++i) {
    const int32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// Stable scatter of one pass (the same wave-rank scheme as the cell sort).
template <typename T>
__global__ void __launch_bounds__(kBlock) radix_scatter_kernel(const T* __restrict__ in, int64_t n, int64_t chunk,
                                                              int pass, const int32_t* __restrict__ base_in,
                                                              T* __restrict__ out) {
  __shared__ int32_t base[256];
  base[threadIdx.x] = base_in[int64_t(threadIdx.x) * gridDim.x + blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = min(n, lo + chunk);
  for (int64_t r0 = lo; r0 < hi; r0 += kBlock) {
    const int64_t i = r0 + threadIdx.x;
    const bool valid = i < hi;
    const T v = valid ? in[i] : T(0);
    const int d = valid ? digit_of(v, pass) : -1;
    int rank = 0, after = 0;
    for (int k = 0; k < 64; ++k) {
      const int dk = __shfl(d, k, 64);
      if (dk == d) {
        if (k < lane) ++rank;
        if (k > lane) ++after;
      }
    }
    for (int w = 0; w < kBlock / 64; ++w) {
      if (wave == w && valid) out[base[d] + rank] = v;
      __syncthreads();
      if (wave == w && valid && after == 0) base[d] += rank + 1;
      __syncthreads();
    }
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

size_t poisson_max_m() { return kMaxFftM; }

__global__ void __launch_bounds__(kBlock) field_energy_kernel(const double* __restrict__ E, int M, double half_dx,
                                                             double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int g = threadIdx.x; g < M; g += kBlock) s = fma(E[g], E[g], s);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    *out = half_dx * t;
  }
}

kde_status launch_field_energy(const double* E, int M, double L, double* out, hipStream_t s) {
  hipLaunchKernelGGL(field_energy_kernel, dim3(1), dim3(kBlock), 0, s, E, M, 0.5 * (L / M), out);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status launch_poisson_field(const double* rho, int M, double L, double* E, double* phi, hipStream_t s) {
  int bits = 0;
  while ((1 << bits) < M) ++bits;
  if ((1 << bits) != M || M > kMaxFftM || M < 2) return fail(KDE_E_INVALID_ARG, "M must be a power of two in [2, %d]", kMaxFftM);
  hipLaunchKernelGGL(poisson_field_kernel, dim3(1), dim3(kBlock), 0, s, rho, M, bits, L, E, phi);
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
  int64_t b = ceil_div(n, 4096);
  if (b < 1) b = 1;
  if (b > 256) b = 256;
  return b;
}

size_t ad_workspace_bytes(int64_t n, int prec) {
  const int64_t blocks = ad_blocks(n);
  const int64_t tb = ceil_div(n, kBlock);
  Carver c(nullptr, 0);
  c.take<char>(size_t(n) * elem_size(prec));
  c.take<char>(size_t(n) * elem_size(prec));
  c.take<int32_t>(256 * size_t(blocks));
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
  double* parts = c.take<double>(size_t(tb));
  double* scratch = c.take<double>(column_sum_scratch(tb, 1) / sizeof(double) + 1);
  double* sum = c.take<double>(1);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "AD workspace too small: %zu < %zu", ws_bytes, c.used);
  KDE_TRY_HIP(hipMemcpyAsync(buf0, x, size_t(n) * sizeof(T), hipMemcpyDeviceToDevice, s));
  T* src = buf0;
  T* dst = buf1;
  for (int pass = 0; pass < KeyOf<T>::passes; ++pass) {
    hipLaunchKernelGGL(radix_hist_kernel<T>, dim3(unsigned(blocks)), dim3(kBlock), 0, s, (const T*)src, n, chunk, pass, hist);
    KDE_CHECK_LAUNCH();
    hipLaunchKernelGGL(radix_scan_kernel, dim3(1), dim3(kBlock), 0, s, hist, int64_t(256) * blocks);
    KDE_CHECK_LAUNCH();
    hipLaunchKernelGGL(radix_scatter_kernel<T>, dim3(unsigned(blocks)), dim3(kBlock), 0, s, (const T*)src, n, chunk, pass,
                       (const int32_t*)hist, dst);
    KDE_CHECK_LAUNCH();
    T* t = src;
    src = dst;
    dst = t;
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
