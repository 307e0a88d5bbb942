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
//
// The first-order (triangular) shape of adjustable width (dev_tri.hpp)
// deposits and gathers with the same decomposition; its per-particle
// parameter is the half-width h_i. Adaptive widths are von Mises only.
#include "dev_density.hpp"
#include "dev_tri.hpp"

namespace kde {

// Dynamic LDS: the node table, M SinCos<T> (2 M values of T).
template <typename T, bool PER, int G>
__global__ void __launch_bounds__(kBlock) deposit_kernel(const T* __restrict__ x, const T* __restrict__ kap,
                                                        double kappa_g, int64_t n, int M, double L, int chunk,
                                                        double* __restrict__ partials, uint32_t* status) {
  __shared__ DepSmem<T> sm;
  extern __shared__ __align__(16) unsigned char dyn[];
  SinCos<T>* tab = reinterpret_cast<SinCos<T>*>(dyn);
  node_table(M, tab);
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int cnt = int(min(int64_t(chunk), n - lo));
  deposit_block<T, PER, G>(x, kap, kappa_g, M, L, lo, cnt, partials + int64_t(blockIdx.x) * M, tab, sm, status);
}

// S adjacent lanes per particle (S = 1, 2, 4 or 8, from gather_split), lane
// j summing the nodes k = j, j + S, j + 2S, ... in order (interleaved, so
// the S lanes read neighbouring LDS words instead of one bank); the S
// partial sums are combined by an xor butterfly, a fixed pairwise tree
// whose result every lane of the group holds. Dynamic LDS: the node table
// (M SinCos<T>) and the field (M values of T). In the float form the loop
// runs over k = g - g0, so the table read is a broadcast and the field read
// is per lane.
template <typename T, int S>
__global__ void __launch_bounds__(kBlock) gather_kernel(const T* __restrict__ x, const T* __restrict__ kap,
                                                       double kappa_g, bool per, int64_t n, int M, double L,
                                                       const double* __restrict__ field, T* __restrict__ out,
                                                       uint32_t* status) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ double etab[std::is_same<T, double>::value ? 256 : 1];
  SinCos<T>* tab = reinterpret_cast<SinCos<T>*>(dyn);
  T* tf = reinterpret_cast<T*>(tab + M);
  exp_table_fill<T>(etab);
  node_table(M, tab);
  for (int k = threadIdx.x; k < M; k += kBlock) tf[k] = T(field[k]);
  __syncthreads();
  const int64_t gid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t i = gid / S;
  if (i >= n) return;  // a particle's S lanes leave together
  const int j = int(gid % S);
  const double xi = double(x[i]);
  const double xw = xi - L * floor(xi / L);
  PGeo<T> gp;
  make_geo(xw, L, M, gp);
  const double kk = per ? double(kap[i]) : kappa_g;
  if (j == 0) note_numeric(status, !isfinite(xi), per && !(isfinite(kk) && kk >= 0.0));
  const T A = T(-2.0 * kk * Flt<T>::unit);
  const double w = (L / M) / (L * i0e_f64(kk));
  Acc<T> acc;
  acc.zero();
  if constexpr (std::is_same<T, float>::value) {
    // node g = g0 + k (mod M); groups of four without a bound test inside
    // a group keep their LDS reads in flight together (the run folds fall
    // after every kRun terms either way)
    auto term = [&](int k) {
      const SinCos<T> e = tab[k];
      const T s = e.s * gp.cb - e.c * gp.sb;
      const int g = gp.g0 + k;
      return tf[g >= M ? g - M : g] * Flt<T>::ex(A * (s * s), etab);
    };
    int k = j, q = 0;
    for (; k + 3 * S < M; k += 4 * S, q += 4) {
      T e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = term(k + u * S);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc.add(e[u]);
      if (((q + 4) & (kRun - 1)) == 0) acc.fold();
    }
    for (; k < M; k += S, ++q) {
      acc.add(term(k));
      if ((q & (kRun - 1)) == kRun - 1) acc.fold();
    }
  } else if (__all(A >= T(-2.0 * kNearKappa))) {
    for (int g = j; g < M; g += S) {
      const T s = node_s(gp, g, M, tab);
      acc.add(tf[g] * Flt<T>::ex_in(A * (s * s), etab));
    }
  } else if (__all(A >= T(kExpTableMin))) {
    // sharp kernels in the wave: near nodes take the exact separation
    const double dx = L / double(M);
    const bool sharp = A < T(-2.0 * kNearKappa);
    for (int g = j; g < M; g += S) {
      T s = node_s(gp, g, M, tab);
      if (sharp) s = near_node_s(s, g, dx, gp.w, L);
      acc.add(tf[g] * Flt<T>::ex_in(A * (s * s), etab));
    }
  } else {
    const double dx = L / double(M);
    const bool sharp = A < T(-2.0 * kNearKappa);
    for (int g = j; g < M; g += S) {
      T s = node_s(gp, g, M, tab);
      if (sharp) s = near_node_s(s, g, dx, gp.w, L);
      acc.add(tf[g] * Flt<T>::ex(A * (s * s), etab));
    }
  }
  double tot = acc.value();
#pragma unroll
  for (int m = 1; m < S; m <<= 1) tot += __shfl_xor(tot, m, 64);
  if (j == 0) out[i] = T(w * tot);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adapt_logsum_kernel(const T* __restrict__ x, int64_t n, int M, double L,
                                                             const double* __restrict__ pilot,
                                                             double* __restrict__ partials, uint32_t* status) {
  __shared__ double r0[kBlock / 64], r1[kBlock / 64];
  adapt_logsum_block<T>(x, n, M, L, pilot, blockIdx.x, partials + 2 * int64_t(blockIdx.x), r0, r1, status);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) adapt_apply_kernel(const T* __restrict__ x, int64_t n, int M, double L,
                                                            const double* __restrict__ pilot, double kappa_star,
                                                            double alpha, const double* __restrict__ sums,
                                                            T* __restrict__ kout, double* __restrict__ log_g_out,
                                                            int64_t* __restrict__ nfl_out) {
  adapt_apply_block<T>(x, n, M, L, pilot, kappa_star, alpha, sums, blockIdx.x, kout);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (log_g_out) *log_g_out = sums[0] / double(n);
    if (nfl_out) *nfl_out = int64_t(sums[1]);
  }
}

// First-order (triangular) shape: the same chunked deposit with triangles
// (dev_tri.hpp), and a gather over the M nodes with the field in LDS.
template <typename T, bool PER, int G>
__global__ void __launch_bounds__(kBlock) tri_deposit_kernel(const T* __restrict__ x, const T* __restrict__ hi,
                                                            double h_g, int64_t n, int M, double L, int chunk,
                                                            double* __restrict__ partials, uint32_t* status) {
  __shared__ TriDepSmem<T> sm;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int cnt = int(min(int64_t(chunk), n - lo));
  tri_deposit_block<T, PER, G>(x, hi, h_g, M, L, lo, cnt, partials + int64_t(blockIdx.x) * M, sm, status);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) tri_gather_kernel(const T* __restrict__ x, const T* __restrict__ hi,
                                                           double h_g, bool per, int64_t n, int M, double L,
                                                           const double* __restrict__ field, T* __restrict__ out,
                                                           uint32_t* status) {
  extern __shared__ __align__(16) unsigned char dyn[];
  T* tf = reinterpret_cast<T*>(dyn);
  for (int k = threadIdx.x; k < M; k += kBlock) tf[k] = T(field[k]);
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double h = per ? double(hi[i]) : h_g;
  note_numeric(status, !isfinite(double(x[i])), per && !(h > 0.0 && h <= 0.5 * L));
  const TriGeo<T> p = tri_geo<T>(double(x[i]), h, L, M);
  // a Kahan step per node: a support spans a few nodes, and runs with their
  // fold test were 15 % slower here in float
  SumOf<T> acc;
  auto add = [&](T v) { acc.add(v); };
  // Nodes beyond h / dx cells of the particle add exact zeros, so a
  // particle whose support is shorter than the circle visits only the nodes
  // g0 - r .. g0 + r (one node of margin against the rounding of q), still
  // in ascending node order: for a finite field the sum is the full
  // loop's, bit for bit.
  const int r = int(fmin(ceil(h * (double(M) / L)), double(M))) + 1;
  if (isfinite(double(p.w)) && 2 * r < M) {
    const int a = p.g0 - r, b = p.g0 + r;
    const int lo1 = a < 0 ? 0 : (b >= M ? 0 : a);
    const int hi1 = a < 0 ? b : (b >= M ? b - M : b);
    const int lo2 = a < 0 ? a + M : (b >= M ? a : M);
    for (int g = lo1; g <= hi1; ++g) add(tf[g] * tri_node(p, g, M));
    for (int g = lo2; g < M; ++g) add(tf[g] * tri_node(p, g, M));
  } else {
    for (int g = 0; g < M; ++g) add(tf[g] * tri_node(p, g, M));
  }
  out[i] = T((L / M) * double(p.w) * acc.value());
}

// ------------------------------------------------------------------ host

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
                                   double* rho, double* partials, int chunk, int64_t chunks, hipStream_t s,
                                   uint32_t* status) {
  const int M = dom->M;
  const dim3 grid{unsigned(chunks)}, block{unsigned(kBlock)};
  const double kg = kappa;
  const size_t lds = 2 * size_t(M) * sizeof(T);
  KDE_RETURN_IF(check_lds(lds + sizeof(DepSmem<T>)));
  TimedLaunch timed(KDE_KERNEL_DEPOSIT, s);
  if (M <= kBlock) {
    hipExtLaunchKernelGGL((deposit_kernel<T, PER, 1>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kg, n, M, dom->L, chunk, partials, status);
  } else if (M <= 2 * kBlock) {
    hipExtLaunchKernelGGL((deposit_kernel<T, PER, 2>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kg, n, M, dom->L, chunk, partials, status);
  } else if (M <= 4 * kBlock) {
    hipExtLaunchKernelGGL((deposit_kernel<T, PER, 4>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kg, n, M, dom->L, chunk, partials, status);
  } else if (M <= 8 * kBlock) {
    hipExtLaunchKernelGGL((deposit_kernel<T, PER, 8>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kg, n, M, dom->L, chunk, partials, status);
  } else {
    hipExtLaunchKernelGGL((deposit_kernel<T, PER, 16>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kg, n, M, dom->L, chunk, partials, status);
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

template <typename T, bool PER>
static kde_status launch_tri_deposit_t(const kde_domain* dom, int64_t n, const T* x, const T* hi, double h,
                                       double* partials, int chunk, int64_t chunks, hipStream_t s,
                                       uint32_t* status) {
  const int M = dom->M;
  const dim3 grid{unsigned(chunks)}, block{unsigned(kBlock)};
  KDE_RETURN_IF(check_lds(sizeof(TriDepSmem<T>)));
  TimedLaunch timed(KDE_KERNEL_DEPOSIT, s);
  if (M <= kBlock) {
    hipExtLaunchKernelGGL((tri_deposit_kernel<T, PER, 1>), grid, block, 0, s, timed.start(), timed.stop(), 0, x, hi, h, n, M, dom->L, chunk, partials, status);
  } else if (M <= 2 * kBlock) {
    hipExtLaunchKernelGGL((tri_deposit_kernel<T, PER, 2>), grid, block, 0, s, timed.start(), timed.stop(), 0, x, hi, h, n, M, dom->L, chunk, partials, status);
  } else if (M <= 4 * kBlock) {
    hipExtLaunchKernelGGL((tri_deposit_kernel<T, PER, 4>), grid, block, 0, s, timed.start(), timed.stop(), 0, x, hi, h, n, M, dom->L, chunk, partials, status);
  } else if (M <= 8 * kBlock) {
    hipExtLaunchKernelGGL((tri_deposit_kernel<T, PER, 8>), grid, block, 0, s, timed.start(), timed.stop(), 0, x, hi, h, n, M, dom->L, chunk, partials, status);
  } else {
    hipExtLaunchKernelGGL((tri_deposit_kernel<T, PER, 16>), grid, block, 0, s, timed.start(), timed.stop(), 0, x, hi, h, n, M, dom->L, chunk, partials, status);
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status deposit(const kde_domain* dom, int64_t n, const void* x, const void* kap, double kappa, double* rho,
                   void* ws, size_t ws_bytes, hipStream_t s, uint32_t* status) {
  const int chunk = deposit_chunk(n);
  const int64_t chunks = ceil_div(n, chunk);
  Carver c(ws, ws_bytes);
  double* partials = c.take<double>(size_t(chunks) * dom->M);
  double* scratch = c.take<double>(column_sum_scratch(chunks, dom->M) / sizeof(double) + 1);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.used);
  if (dom->shape == KDE_SHAPE_TRIANGLE) {
    if (dom->prec == KDE_F64) {
      const double* xx = static_cast<const double*>(x);
      const double* hh = static_cast<const double*>(kap);
      KDE_RETURN_IF((hh ? launch_tri_deposit_t<double, true>(dom, n, xx, hh, kappa, partials, chunk, chunks, s, status)
                        : launch_tri_deposit_t<double, false>(dom, n, xx, hh, kappa, partials, chunk, chunks, s, status)));
    } else {
      const float* xx = static_cast<const float*>(x);
      const float* hh = static_cast<const float*>(kap);
      KDE_RETURN_IF((hh ? launch_tri_deposit_t<float, true>(dom, n, xx, hh, kappa, partials, chunk, chunks, s, status)
                        : launch_tri_deposit_t<float, false>(dom, n, xx, hh, kappa, partials, chunk, chunks, s, status)));
    }
  } else if (dom->prec == KDE_F64) {
    const double* xx = static_cast<const double*>(x);
    const double* kk = static_cast<const double*>(kap);
    KDE_RETURN_IF((kk ? launch_deposit_t<double, true>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s, status)
                      : launch_deposit_t<double, false>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s, status)));
  } else {
    const float* xx = static_cast<const float*>(x);
    const float* kk = static_cast<const float*>(kap);
    KDE_RETURN_IF((kk ? launch_deposit_t<float, true>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s, status)
                      : launch_deposit_t<float, false>(dom, n, xx, kk, kappa, rho, partials, chunk, chunks, s, status)));
  }
  return launch_column_sum(partials, chunks, dom->M, scratch, rho, s, 1.0 / double(n));
}

// Lanes per particle for the gather: split the node loop while the
// particles alone would leave the chip short of workgroups (fewer than
// 1024) and every lane keeps at least 32 nodes.
static int gather_split(int64_t n, int M) {
  int S = 1;
  while (S < 8 && M / (2 * S) >= 32 && ceil_div(n * S, kBlock) < 1024) S *= 2;
  return S;
}

template <typename T>
static kde_status launch_gather_t(const kde_domain* dom, int64_t n, const T* x, const T* kap, double kappa,
                                  const double* field, T* out, size_t lds, hipStream_t s, uint32_t* status) {
  const int S = gather_split(n, dom->M);
  const dim3 grid{unsigned(ceil_div(n * S, kBlock))}, block{unsigned(kBlock)};
  const bool per = kap != nullptr;
  TimedLaunch timed(KDE_KERNEL_GATHER, s);
  switch (S) {
    case 1:
      hipExtLaunchKernelGGL((gather_kernel<T, 1>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kappa, per, n, dom->M, dom->L, field, out, status);
      break;
    case 2:
      hipExtLaunchKernelGGL((gather_kernel<T, 2>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kappa, per, n, dom->M, dom->L, field, out, status);
      break;
    case 4:
      hipExtLaunchKernelGGL((gather_kernel<T, 4>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kappa, per, n, dom->M, dom->L, field, out, status);
      break;
    default:
      hipExtLaunchKernelGGL((gather_kernel<T, 8>), grid, block, lds, s, timed.start(), timed.stop(), 0, x, kap, kappa, per, n, dom->M, dom->L, field, out, status);
      break;
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status gather(const kde_domain* dom, int64_t n, const void* x, const void* kap, double kappa,
                  const double* field, void* out, hipStream_t s, uint32_t* status) {
  const dim3 grid{unsigned(ceil_div(n, kBlock))}, block{unsigned(kBlock)};
  if (dom->shape == KDE_SHAPE_TRIANGLE) {
    const size_t lds = size_t(dom->M) * elem_size(dom->prec);
    KDE_RETURN_IF(check_lds(lds));
    TimedLaunch timed(KDE_KERNEL_GATHER, s);
    if (dom->prec == KDE_F64)
      hipExtLaunchKernelGGL(tri_gather_kernel<double>, grid, block, lds, s, timed.start(), timed.stop(), 0,
                         static_cast<const double*>(x),
                         static_cast<const double*>(kap), kappa, kap != nullptr, n, dom->M, dom->L, field,
                         static_cast<double*>(out), status);
    else
      hipExtLaunchKernelGGL(tri_gather_kernel<float>, grid, block, lds, s, timed.start(), timed.stop(), 0,
                         static_cast<const float*>(x),
                         static_cast<const float*>(kap), kappa, kap != nullptr, n, dom->M, dom->L, field,
                         static_cast<float*>(out), status);
    KDE_CHECK_LAUNCH();
    return KDE_OK;
  }
  const size_t lds = 3 * size_t(dom->M) * elem_size(dom->prec);
  KDE_RETURN_IF(check_lds(lds + (dom->prec == KDE_F64 ? 256 * sizeof(double) : sizeof(double))));  // + exp table
  if (dom->prec == KDE_F64)
    KDE_RETURN_IF(launch_gather_t<double>(dom, n, static_cast<const double*>(x), static_cast<const double*>(kap),
                                          kappa, field, static_cast<double*>(out), lds, s, status));
  else
    KDE_RETURN_IF(launch_gather_t<float>(dom, n, static_cast<const float*>(x), static_cast<const float*>(kap),
                                         kappa, field, static_cast<float*>(out), lds, s, status));
  return KDE_OK;
}

kde_status adapt_widths(const kde_domain* dom, int64_t n, const void* x, const double* pilot, double kappa_star,
                        double alpha, void* kout, double* log_g, int64_t* nfl, void* ws, size_t ws_bytes,
                        hipStream_t s, uint32_t* status) {
  const int64_t blocks = ceil_div(n, kBlock);
  Carver c(ws, ws_bytes);
  double* partials = c.take<double>(size_t(blocks) * 2);
  double* scratch = c.take<double>(column_sum_scratch(blocks, 2) / sizeof(double) + 1);
  double* sums = c.take<double>(2);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.used);
  const dim3 grid{unsigned(blocks)}, block{unsigned(kBlock)};
  TimedLaunch timed(KDE_KERNEL_ADAPT, s);  // from the log sums' start to the widths' end
  if (dom->prec == KDE_F64) {
    hipExtLaunchKernelGGL(adapt_logsum_kernel<double>, grid, block, 0, s, timed.start(), nullptr, 0,
                          static_cast<const double*>(x), n, dom->M, dom->L, pilot, partials, status);
  } else {
    hipExtLaunchKernelGGL(adapt_logsum_kernel<float>, grid, block, 0, s, timed.start(), nullptr, 0,
                          static_cast<const float*>(x), n, dom->M, dom->L, pilot, partials, status);
  }
  KDE_CHECK_LAUNCH();
  KDE_RETURN_IF(launch_column_sum(partials, blocks, 2, scratch, sums, s));
  if (dom->prec == KDE_F64) {
    hipExtLaunchKernelGGL(adapt_apply_kernel<double>, grid, block, 0, s, nullptr, timed.stop(), 0,
                          static_cast<const double*>(x), n, dom->M, dom->L, pilot, kappa_star, alpha,
                          (const double*)sums, static_cast<double*>(kout), log_g, nfl);
  } else {
    hipExtLaunchKernelGGL(adapt_apply_kernel<float>, grid, block, 0, s, nullptr, timed.stop(), 0,
                          static_cast<const float*>(x), n, dom->M, dom->L, pilot, kappa_star, alpha,
                          (const double*)sums, static_cast<float*>(kout), log_g, nfl);
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

}  // namespace kde
