// Grid density, field gather and adaptive widths with von Mises kernels.
//
// Deposit (Sec. II.B Eq. kde; Sec. II.C step 3 for per-particle widths):
//   rho[g] = (1/N) sum_i w_i exp(-2 kappa_i s_ig^2),
//   s_ig = sin(pi (x_g - x_i) / L),  w_i = 1 / (L I0e(kappa_i)).
// The grid is small (M <= 4096) and every particle touches every node, so
// a workgroup owns the whole grid for one contiguous chunk of particles:
// the chunk is staged in LDS (half-angle vector, exponent scale, weight)
// and read by all lanes at the same address (broadcast), each thread
// accumulating its own node(s). Per-chunk grids go to fixed slots and are
// summed in a fixed order. The cost is one exponential per (particle, node):
// transcendental-bound, not HBM-bound, at every grid size used here.
//
// Gather (field interpolation of Sec. III.A with the same kernels):
//   out[i] = (L/M) w_i sum_g F_g exp(-2 kappa_i s_ig^2),
// one thread per particle with the node table in LDS.
//
// Adaptive widths (Sec. II.C, Eq. adaptive_width): the pilot grid is
// interpolated linearly at each particle, its logarithms are averaged in
// double (fixed-order reduction), and kappa_i = kappa* exp(2 alpha (log f_i
// - log g)) is written per particle.
#include <cfloat>

#include "device_bessel.hpp"
#include "kde_internal.hpp"

namespace kde {

template <typename T>
struct Flt;
template <>
struct Flt<double> {
  static __device__ __forceinline__ double ex(double a) { return exp(a); }  // a = natural exponent
  static constexpr double unit = 1.0;
  static constexpr double tiny = DBL_MIN;
};
template <>
struct Flt<float> {
  static __device__ __forceinline__ float ex(float a) { return __builtin_amdgcn_exp2f(a); }  // base 2
  static constexpr double unit = 1.4426950408889634;
  static constexpr float tiny = FLT_MIN;
};

template <typename T>
struct SumOf;
template <>
struct SumOf<double> {
  double s = 0.0;
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ double value() const { return s; }
};
template <>
struct SumOf<float> {
  float s = 0.0f, c = 0.0f;
  __device__ __forceinline__ void add(float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const { return double(s) - double(c); }
};

constexpr int kDepMaxChunk = 512;

// Geometry of a (node, particle) pair. Both forms give s = sin(pi (x_g - x_i) / L):
//   double: global half-angle vectors, s = sin(pi g/M) a_i - cos(pi g/M) b_i with
//           (a_i, b_i) = (cos(pi x_i/L), sin(pi x_i/L));
//   float : node-relative, with the particle at v = x_i M / L split as v = g0 + d
//           (g0 the nearest node, |d| <= 1/2) and beta = pi d / M:
//           s = sin(pi k/M) cos(beta) - cos(pi k/M) sin(beta), k = (g - g0) mod M,
//           from a table over k. Near nodes have small k and small beta, so s
//           keeps float relative accuracy where the kernel is largest (the
//           global form would carry the absolute rounding of a_i, b_i).
template <typename T>
struct PGeo;
template <>
struct PGeo<double> {
  double a, b;
};
template <>
struct PGeo<float> {
  int g0;
  float cb, sb;
};

__device__ __forceinline__ void make_geo(double xw, double L, int M, PGeo<double>& p) {
  double sp, cp;
  sincospi(xw / L, &sp, &cp);
  p.a = cp;
  p.b = sp;
}

__device__ __forceinline__ void make_geo(double xw, double L, int M, PGeo<float>& p) {
  const double v = xw * (double(M) / L);
  double g0 = floor(v + 0.5);
  const double d = v - g0;
  if (g0 >= double(M)) g0 -= double(M);
  double sb, cb;
  sincospi(d / double(M), &sb, &cb);
  p.g0 = int(g0);
  p.cb = float(cb);
  p.sb = float(sb);
}

template <typename T, bool PER>
__device__ __forceinline__ void particle_terms(const T* __restrict__ x, const T* __restrict__ kap, double kappa_g,
                                               int64_t i, double L, int M, PGeo<T>& g, T& A, T& w) {
  const double xi = double(x[i]);
  const double xw = xi - L * floor(xi / L);
  make_geo(xw, L, M, g);
  const double k = PER ? double(kap[i]) : kappa_g;
  A = T(-2.0 * k * Flt<T>::unit);
  w = PER ? T(1.0 / (L * i0e_f64(k))) : T(1);
}

// s for node g of a particle; `ts`/`tc` hold sin/cos(pi g/M) (double form,
// indexed by g) or sin/cos(pi k/M) (float form, indexed by k = g - g0 mod M).
__device__ __forceinline__ double node_s(const PGeo<double>& p, int g, int M, const double* ts, const double* tc) {
  return ts[g] * p.a - tc[g] * p.b;
}
__device__ __forceinline__ float node_s(const PGeo<float>& p, int g, int M, const float* ts, const float* tc) {
  int k = g - p.g0;
  k += (k < 0) ? M : 0;
  return ts[k] * p.cb - tc[k] * p.sb;
}

// One workgroup: particles [blk*chunk, ...), all M nodes.
// M <= 256: S = 256 / M sub-streams share a node, thread t -> node t % M,
//           sub-stream t / M (threads beyond S*M idle);
// M  > 256: thread t -> nodes t, t + 256, ... (G per thread).
// Dynamic LDS: the node table, 2 M values of T.
template <typename T, bool PER, int G>
__global__ void __launch_bounds__(kBlock) deposit_kernel(const T* __restrict__ x, const T* __restrict__ kap,
                                                        double kappa_g, int64_t n, int M, double L, int chunk,
                                                        double* __restrict__ partials) {
  __shared__ PGeo<T> pg[kDepMaxChunk];
  __shared__ T pA[kDepMaxChunk], pw[kDepMaxChunk];
  __shared__ double red[kBlock];
  extern __shared__ __align__(16) unsigned char dyn[];
  T* ts = reinterpret_cast<T*>(dyn);
  T* tc = ts + M;
  const int tid = threadIdx.x;
  for (int k = tid; k < M; k += kBlock) {
    double sv, cv;
    sincospi(double(k) / double(M), &sv, &cv);
    ts[k] = T(sv);
    tc[k] = T(cv);
  }
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int cnt = int(min(int64_t(chunk), n - lo));
  for (int k = tid; k < cnt; k += kBlock) particle_terms<T, PER>(x, kap, kappa_g, lo + k, L, M, pg[k], pA[k], pw[k]);
  __syncthreads();
  double* out = partials + int64_t(blockIdx.x) * M;
  if (M <= kBlock) {
    const int S = kBlock / M;
    const int g = tid % M, sub = tid / M;
    double tot = 0.0;
    if (sub < S) {
      SumOf<T> acc;
      for (int p = sub; p < cnt; p += S) {
        const T s = node_s(pg[p], g, M, ts, tc);
        const T e = Flt<T>::ex(pA[p] * (s * s));
        acc.add(PER ? pw[p] * e : e);
      }
      tot = acc.value();
    }
    red[tid] = tot;
    __syncthreads();
    if (tid < M) {
      double v = 0.0;
      for (int q = 0; q < S; ++q) v += red[q * M + tid];
      out[tid] = PER ? v : v * (1.0 / (L * i0e_f64(kappa_g)));
    }
  } else {
    SumOf<T> acc[G];
    for (int p = 0; p < cnt; ++p) {
      const PGeo<T> gp = pg[p];
      const T A = pA[p], w = pw[p];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int g = tid + k * kBlock;
        if (g < M) {
          const T s = node_s(gp, g, M, ts, tc);
          const T e = Flt<T>::ex(A * (s * s));
          acc[k].add(PER ? w * e : e);
        }
      }
    }
    const double scale = PER ? 1.0 : 1.0 / (L * i0e_f64(kappa_g));
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = tid + k * kBlock;
      if (g < M) out[g] = acc[k].value() * scale;
    }
  }
}

// One thread per particle, looping over the nodes. Dynamic LDS: the node
// table (2 M values of T) and the field (M values of T). In the float form
// the loop runs over k = g - g0, so the table read is a broadcast and the
// field read is per lane.
template <typename T>
__global__ void __launch_bounds__(kBlock) gather_kernel(const T* __restrict__ x, const T* __restrict__ kap,
                                                       double kappa_g, bool per, int64_t n, int M, double L,
                                                       const double* __restrict__ field, T* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char dyn[];
  T* ts = reinterpret_cast<T*>(dyn);
  T* tc = ts + M;
  T* tf = tc + M;
  for (int k = threadIdx.x; k < M; k += kBlock) {
    double sv, cv;
    sincospi(double(k) / double(M), &sv, &cv);
    ts[k] = T(sv);
    tc[k] = T(cv);
    tf[k] = T(field[k]);
  }
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double xi = double(x[i]);
  const double xw = xi - L * floor(xi / L);
  PGeo<T> gp;
  make_geo(xw, L, M, gp);
  const double kk = per ? double(kap[i]) : kappa_g;
  const T A = T(-2.0 * kk * Flt<T>::unit);
  const double w = (L / M) / (L * i0e_f64(kk));
  SumOf<T> acc;
  if constexpr (std::is_same<T, float>::value) {
    int g = gp.g0;
    for (int k = 0; k < M; ++k) {
      const T s = ts[k] * gp.cb - tc[k] * gp.sb;
      acc.add(tf[g] * Flt<T>::ex(A * (s * s)));
      g = (g + 1 == M) ? 0 : g + 1;
    }
  } else {
    for (int g = 0; g < M; ++g) {
      const T s = node_s(gp, g, M, ts, tc);
      acc.add(tf[g] * Flt<T>::ex(A * (s * s)));
    }
  }
  out[i] = T(w * acc.value());
}

// ------------------------------------------------------------------ adapt

// Pilot density at a particle: periodic linear interpolation between the
// two nodes around it, floored at the smallest normal number of T. A
// non-finite position yields NaN (and is not counted as floored). The
// arithmetic is double in both precisions: this step reads and writes a
// few bytes per particle and is bound by memory traffic, not arithmetic.
template <typename T>
__device__ __forceinline__ double pilot_at(T xv, double L, int M, const double* __restrict__ pilot, bool& floored) {
  const double xi = double(xv);
  floored = false;
  if (!isfinite(xi)) return NAN;
  const double xw = xi - L * floor(xi / L);
  double u = xw * (double(M) / L);
  if (!(u >= 0.0)) u = 0.0;
  int j = int(floor(u));
  double t = u - double(j);
  if (j >= M) {  // x rounded up to L: the node at 0
    j = 0;
    t = 0.0;
  }
  const int j1 = (j + 1 == M) ? 0 : j + 1;
  double f = (1.0 - t) * pilot[j] + t * pilot[j1];
  if (f < double(Flt<T>::tiny)) {  // NaN stays NaN
    floored = true;
    f = double(Flt<T>::tiny);
  }
  return f;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adapt_logsum_kernel(const T* __restrict__ x, int64_t n, int M, double L,
                                                             const double* __restrict__ pilot,
                                                             double* __restrict__ partials) {
  __shared__ double r0[kBlock / 64], r1[kBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  double lsum = 0.0, fl = 0.0;
  if (i < n) {
    bool floored;
    lsum = log(pilot_at<T>(x[i], L, M, pilot, floored));
    fl = floored ? 1.0 : 0.0;
  }
  lsum = wave_sum(lsum);
  fl = wave_sum(fl);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    r0[wave] = lsum;
    r1[wave] = fl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      a += r0[w];
      b += r1[w];
    }
    partials[2 * int64_t(blockIdx.x)] = a;
    partials[2 * int64_t(blockIdx.x) + 1] = b;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adapt_apply_kernel(const T* __restrict__ x, int64_t n, int M, double L,
                                                            const double* __restrict__ pilot, double kappa_star,
                                                            double alpha, const double* __restrict__ sums,
                                                            T* __restrict__ kout, double* __restrict__ log_g_out,
                                                            int64_t* __restrict__ nfl_out) {
  const double log_g = sums[0] / double(n);
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) {
    bool floored;
    const double lf = log(pilot_at<T>(x[i], L, M, pilot, floored));
    kout[i] = T(kappa_star * exp(2.0 * alpha * (lf - log_g)));
  }
  if (i == 0) {
    if (log_g_out) *log_g_out = log_g;
    if (nfl_out) *nfl_out = int64_t(sums[1]);
  }
}

// ------------------------------------------------------------------ host

static int deposit_chunk(int64_t n) {
  int64_t c = ceil_div(n, 2048);
  if (c < 64) c = 64;
  if (c > kDepMaxChunk) c = kDepMaxChunk;
  return int(c);
}

size_t deposit_workspace_bytes(int64_t n, int M) {
  const int64_t chunks = ceil_div(n, deposit_chunk(n));
  Carver c(nullptr, 0);
  c.take<double>(size_t(chunks) * M);
  c.take<double>(column_sum_scratch(chunks, M) / sizeof(double) + 1);
  return c.used;
}

size_t adapt_workspace_bytes(int64_t n) {
  const int64_t blocks = ceil_div(n, kBlock);
  Carver c(nullptr, 0);
  c.take<double>(size_t(blocks) * 2);
  c.take<double>(column_sum_scratch(blocks, 2) / sizeof(double) + 1);
  c.take<double>(2);
  return c.used;
}

template <typename T, bool PER>
static kde_status launch_deposit_t(const kde_domain* dom, int64_t n, const T* x, const T* kap, double kappa,
                                   double* rho, double* partials, int chunk, int64_t chunks, hipStream_t s) {
  const int M = dom->M;
  const dim3 grid{unsigned(chunks)}, block{unsigned(kBlock)};
  const double kg = kappa;
  const size_t lds = 2 * size_t(M) * sizeof(T);
  KDE_RETURN_IF(check_lds(lds + kDepMaxChunk * (sizeof(PGeo<T>) + 2 * sizeof(T)) + kBlock * sizeof(double)));
  TimedLaunch timed(KDE_KERNEL_DEPOSIT, s);
  if (M <= kBlock) {
    hipLaunchKernelGGL((deposit_kernel<T, PER, 1>), grid, block, lds, s, x, kap, kg, n, M, dom->L, chunk, partials);
  } else if (M <= 2 * kBlock) {
    hipLaunchKernelGGL((deposit_kernel<T, PER, 2>), grid, block, lds, s, x, kap, kg, n, M, dom->L, chunk, partials);
  } else if (M <= 4 * kBlock) {
    hipLaunchKernelGGL((deposit_kernel<T, PER, 4>), grid, block, lds, s, x, kap, kg, n, M, dom->L, chunk, partials);
  } else if (M <= 8 * kBlock) {
    hipLaunchKernelGGL((deposit_kernel<T, PER, 8>), grid, block, lds, s, x, kap, kg, n, M, dom->L, chunk, partials);
  } else {
    hipLaunchKernelGGL((deposit_kernel<T, PER, 16>), grid, block, lds, s, x, kap, kg, n, M, dom->L, chunk, partials);
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status deposit(const kde_domain* dom, int64_t n, const void* x, const void* kap, double kappa, double* rho,
                   void* ws, size_t ws_bytes, hipStream_t s) {
  const int chunk = deposit_chunk(n);
  const int64_t chunks = ceil_div(n, chunk);
  Carver c(ws, ws_bytes);
  double* partials = c.take<double>(size_t(chunks) * dom->M);
  double* scratch = c.take<double>(column_sum_scratch(chunks, dom->M) / sizeof(double) + 1);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.used);
  if (dom->prec == KDE_F64) {
    const double* xx = static_cast<const double*>(x);
    const double* kk = static_cast<const double*>(kap);
    KDE_RETURN_IF((kk ? launch_deposit_t<double, true>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s)
                      : launch_deposit_t<double, false>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s)));
  } else {
    const float* xx = static_cast<const float*>(x);
    const float* kk = static_cast<const float*>(kap);
    KDE_RETURN_IF((kk ? launch_deposit_t<float, true>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s)
                      : launch_deposit_t<float, false>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s)));
  }
  return launch_column_sum(partials, chunks, dom->M, scratch, rho, s, 1.0 / double(n));
}

kde_status gather(const kde_domain* dom, int64_t n, const void* x, const void* kap, double kappa,
                  const double* field, void* out, hipStream_t s) {
  const dim3 grid{unsigned(ceil_div(n, kBlock))}, block{unsigned(kBlock)};
  const size_t lds = 3 * size_t(dom->M) * elem_size(dom->prec);
  KDE_RETURN_IF(check_lds(lds));
  TimedLaunch timed(KDE_KERNEL_GATHER, s);
  if (dom->prec == KDE_F64) {
    hipLaunchKernelGGL(gather_kernel<double>, grid, block, lds, s, static_cast<const double*>(x),
                       static_cast<const double*>(kap), kappa, kap != nullptr, n, dom->M, dom->L, field,
                       static_cast<double*>(out));
  } else {
    hipLaunchKernelGGL(gather_kernel<float>, grid, block, lds, s, static_cast<const float*>(x),
                       static_cast<const float*>(kap), kappa, kap != nullptr, n, dom->M, dom->L, field,
                       static_cast<float*>(out));
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status adapt_widths(const kde_domain* dom, int64_t n, const void* x, const double* pilot, double kappa_star,
                        double alpha, void* kout, double* log_g, int64_t* nfl, void* ws, size_t ws_bytes,
                        hipStream_t s) {
  const int64_t blocks = ceil_div(n, kBlock);
  Carver c(ws, ws_bytes);
  double* partials = c.take<double>(size_t(blocks) * 2);
  double* scratch = c.take<double>(column_sum_scratch(blocks, 2) / sizeof(double) + 1);
  double* sums = c.take<double>(2);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.used);
  const dim3 grid{unsigned(blocks)}, block{unsigned(kBlock)};
  TimedLaunch timed(KDE_KERNEL_ADAPT, s);
  if (dom->prec == KDE_F64) {
    hipLaunchKernelGGL(adapt_logsum_kernel<double>, grid, block, 0, s, static_cast<const double*>(x), n, dom->M,
                       dom->L, pilot, partials);
  } else {
    hipLaunchKernelGGL(adapt_logsum_kernel<float>, grid, block, 0, s, static_cast<const float*>(x), n, dom->M,
                       dom->L, pilot, partials);
  }
  KDE_CHECK_LAUNCH();
  KDE_RETURN_IF(launch_column_sum(partials, blocks, 2, scratch, sums, s));
  if (dom->prec == KDE_F64) {
    hipLaunchKernelGGL(adapt_apply_kernel<double>, grid, block, 0, s, static_cast<const double*>(x), n, dom->M,
                       dom->L, pilot, kappa_star, alpha, (const double*)sums, static_cast<double*>(kout), log_g,
                       nfl);
  } else {
    hipLaunchKernelGGL(adapt_apply_kernel<float>, grid, block, 0, s, static_cast<const float*>(x), n, dom->M,
                       dom->L, pilot, kappa_star, alpha, (const double*)sums, static_cast<float*>(kout), log_g,
                       nfl);
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

}  // namespace kde
