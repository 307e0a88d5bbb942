// Batching form: many independent particle sets through the whole plain
// path (CV scan over a shared list of concentrations, pilot deposit at each
// set's kappa*, adaptive widths, adaptive deposit) in one hipGraph launch.
//
// The graph holds one persistent kernel per phase. Each kernel runs about
// as many workgroups as the device keeps resident and they pull work units
// -- (set), (set, tile pair), (set, particle chunk) or (set, row block) --
// from the phase's own device counter, sets ordered by decreasing cost so
// that the long pair-sum work starts first. Phases follow each other in
// the graph, so no workgroup ever waits on another. Every unit runs the
// same device code as the one-set entry points and writes its own slot,
// and every reduction has the one-set entry points' fixed order, so each
// set's results are bitwise identical to running it alone.
#include <algorithm>
#include <memory>
#include <numeric>
#include <vector>

#include "dev_cv.hpp"
#include "dev_density.hpp"
#include "dev_layout.hpp"
#include "dev_reduce.hpp"
#include "batch_internal.hpp"
#include <cstring>

namespace kde {

// Phase counters (zeroed by the first kernel of every launch).
enum Phase {
  PH_PACK, PH_CV_L1, PH_CV_FIN, PH_PIL_DEP, PH_PIL_L1, PH_PIL_L2, PH_AD_LOG, PH_AD_L1, PH_AD_L2,
  PH_AD_APPLY, PH_RHO_DEP, PH_RHO_L1, PH_RHO_L2, PH_COUNT
};
// The pair phase runs once per pass-size bucket, bucket k on counter
// PH_COUNT + k.
constexpr int kMaxBuckets = 64;
constexpr int kCounters = PH_COUNT + kMaxBuckets;

// Per-set description as the kernels see it (lives in the workspace).
struct SetDev {
  int64_t n;
  int64_t n_cv;  // particles the CV scan uses (a prefix)
  const void* x;
  double L;
  int M, cells, chunk, pad;
  int64_t units, g_cv, chunks, g_dep, blocks, g_ad;
  void* packed;
  double* partials;   // units x 2B
  double* cv_l1;      // g_cv x 2B
  double* dep_part;   // chunks x M (pilot, then adaptive)
  double* dep_l1;     // g_dep x M
  double* pilot;      // M
  double* ad_part;    // blocks x 2
  double* ad_l1;      // g_ad x 2
  double* ad_sums;    // 2
  void* kappa_i;      // N (prec)
  double* rho;        // M
  double* cv;         // B or NULL
  double* kstar;      // 1
  double* kstar_user; // 1 or NULL
};

// Unit prefix sums, one array of nsets + 1 per multi-unit phase.
enum Prefix { PF_PAIRS, PF_CV_L1, PF_CHUNKS, PF_DEP_L1, PF_BLOCKS, PF_AD_L1, PF_COUNT };

struct BatchArgs {
  const SetDev* sets;
  const int64_t* prefix;  // PF_COUNT x (nsets + 1)
  unsigned long long* counters;
  int nsets;
  int B;
  double alpha;
};

__device__ __forceinline__ int find_set(const int64_t* pf, int nsets, int64_t u) {
  int lo = 0, hi = nsets - 1;  // largest s with pf[s] <= u
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pf[mid] <= u) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Claim the next unit of a phase for the whole workgroup.
__device__ __forceinline__ int64_t claim(unsigned long long* counter, int64_t* slot) {
  if (threadIdx.x == 0) *slot = int64_t(atomicAdd(counter, 1ull));
  __syncthreads();
  const int64_t u = *slot;
  __syncthreads();
  return u;
}

__global__ void __launch_bounds__(kBlock) batch_zero_kernel(unsigned long long* counters) {
  if (threadIdx.x < kCounters) counters[threadIdx.x] = 0ull;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) batch_pack_kernel(BatchArgs a) {
  using P = typename Packed<T>::type;
  __shared__ int64_t slot;
  __shared__ int tot[kBlock];
  extern __shared__ int base[];
  for (;;) {
    const int64_t u = claim(&a.counters[PH_PACK], &slot);
    if (u >= a.nsets) break;
    const SetDev& s = a.sets[u];
    sort_set_one_block<T, P>(static_cast<const T*>(s.x), s.n_cv, s.L, s.cells, base, tot, static_cast<P*>(s.packed));
    __syncthreads();
  }
}

// Pair units [u_lo, u_hi) of the flattened list (one pass-size bucket).
template <typename T, int BC>
__global__ void __launch_bounds__(kBlock) batch_pairs_kernel(BatchArgs a, CvConsts<T> K, int phase, int64_t u_lo,
                                                            int64_t u_hi) {
  using P = typename Packed<T>::type;
  __shared__ int64_t slot;
  __shared__ CvSmem<T, BC> sm;
  const int64_t* pf = a.prefix + PF_PAIRS * (a.nsets + 1);
  for (;;) {
    const int64_t u = u_lo + claim(&a.counters[phase], &slot);
    if (u >= u_hi) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int64_t p = u - pf[si];
    int I, J;
    tri_decode(p, I, J);
    cv_tile_pair<T, BC>(static_cast<const P*>(s.packed), s.n_cv, I, J, K, s.partials + p * 2 * K.B, sm);
  }
}

// Level-1 row blocks of a [rows x cols] partial array of every set.
enum L1Source { SRC_CV, SRC_DEP, SRC_AD };

template <int SRC>
__global__ void __launch_bounds__(kBlock) batch_level1_kernel(BatchArgs a, int phase, int pf_index) {
  __shared__ int64_t slot;
  const int64_t* pf = a.prefix + pf_index * (a.nsets + 1);
  const int64_t total = pf[a.nsets];
  for (;;) {
    const int64_t u = claim(&a.counters[phase], &slot);
    if (u >= total) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int64_t b = u - pf[si];
    const double* in;
    double* l1;
    int64_t rows;
    int cols;
    if (SRC == SRC_CV) {
      in = s.partials; l1 = s.cv_l1; rows = s.units; cols = 2 * a.B;
    } else if (SRC == SRC_DEP) {
      in = s.dep_part; l1 = s.dep_l1; rows = s.chunks; cols = s.M;
    } else {
      in = s.ad_part; l1 = s.ad_l1; rows = s.blocks; cols = 2;
    }
    for (int c = threadIdx.x; c < cols; c += kBlock) l1[b * cols + c] = colsum_level1(in, rows, cols, b, c);
  }
}

// One set per unit: the CV objective from its level-1 rows, argmin, kappa*.
__global__ void __launch_bounds__(kBlock) batch_cv_finalize_kernel(BatchArgs a, KappaList kap) {
  __shared__ int64_t slot;
  __shared__ double raw[2 * KDE_MAX_KAPPAS];
  __shared__ double v[KDE_MAX_KAPPAS];
  __shared__ int best;
  for (;;) {
    const int64_t u = claim(&a.counters[PH_CV_FIN], &slot);
    if (u >= a.nsets) break;
    const SetDev& s = a.sets[u];
    for (int c = threadIdx.x; c < 2 * a.B; c += kBlock) raw[c] = colsum_level2(s.cv_l1, s.g_cv, 2 * a.B, c, 1.0);
    __syncthreads();
    cv_finalize_block(raw, a.B, double(s.n_cv), s.L, kap, s.cv, nullptr, nullptr, v, &best);
    if (threadIdx.x == 0) {
      *s.kstar = kap.k[best];
      if (s.kstar_user) *s.kstar_user = kap.k[best];
    }
    __syncthreads();
  }
}

// Deposit chunks of every set: the pilot at kappa* (PER = false) or the
// adaptive deposit with the set's kappa_i (PER = true).
template <typename T, bool PER, int G>
__global__ void __launch_bounds__(kBlock) batch_deposit_kernel(BatchArgs a, int phase) {
  __shared__ int64_t slot;
  __shared__ DepSmem<T> sm;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int64_t* pf = a.prefix + PF_CHUNKS * (a.nsets + 1);
  const int64_t total = pf[a.nsets];
  T* ts = reinterpret_cast<T*>(dyn);
  for (;;) {
    const int64_t u = claim(&a.counters[phase], &slot);
    if (u >= total) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int64_t c = u - pf[si];
    T* tc = ts + s.M;
    node_table(s.M, ts, tc);
    const int64_t lo = c * s.chunk;
    const int cnt = int(min(int64_t(s.chunk), s.n - lo));
    deposit_block<T, PER, G>(static_cast<const T*>(s.x), static_cast<const T*>(s.kappa_i), PER ? 0.0 : *s.kstar,
                             s.M, s.L, lo, cnt, s.dep_part + c * s.M, ts, tc, sm);
  }
}

// Level 2 of every set: the pilot (scaled by 1/N), the log sums, or rho.
template <int WHAT>  // 0 pilot, 1 adapt sums, 2 rho
__global__ void __launch_bounds__(kBlock) batch_level2_kernel(BatchArgs a, int phase) {
  __shared__ int64_t slot;
  for (;;) {
    const int64_t u = claim(&a.counters[phase], &slot);
    if (u >= a.nsets) break;
    const SetDev& s = a.sets[u];
    if (WHAT == 1) {
      for (int c = threadIdx.x; c < 2; c += kBlock) s.ad_sums[c] = colsum_level2(s.ad_l1, s.g_ad, 2, c, 1.0);
    } else {
      double* out = (WHAT == 0) ? s.pilot : s.rho;
      const double scale = 1.0 / double(s.n);
      for (int c = threadIdx.x; c < s.M; c += kBlock) out[c] = colsum_level2(s.dep_l1, s.g_dep, s.M, c, scale);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) batch_adapt_log_kernel(BatchArgs a) {
  __shared__ int64_t slot;
  __shared__ double r0[kBlock / 64], r1[kBlock / 64];
  const int64_t* pf = a.prefix + PF_BLOCKS * (a.nsets + 1);
  const int64_t total = pf[a.nsets];
  for (;;) {
    const int64_t u = claim(&a.counters[PH_AD_LOG], &slot);
    if (u >= total) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int64_t b = u - pf[si];
    adapt_logsum_block<T>(static_cast<const T*>(s.x), s.n, s.M, s.L, s.pilot, b, s.ad_part + 2 * b, r0, r1);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) batch_adapt_apply_kernel(BatchArgs a) {
  __shared__ int64_t slot;
  const int64_t* pf = a.prefix + PF_BLOCKS * (a.nsets + 1);
  const int64_t total = pf[a.nsets];
  for (;;) {
    const int64_t u = claim(&a.counters[PH_AD_APPLY], &slot);
    if (u >= total) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int64_t b = u - pf[si];
    adapt_apply_block<T>(static_cast<const T*>(s.x), s.n, s.M, s.L, s.pilot, *s.kstar, a.alpha, s.ad_sums, b,
                         static_cast<T*>(s.kappa_i));
  }
}

// ------------------------------------------------------------------ host

// Lay out the workspace; with ws == nullptr only sizes it. Fills host
// images of the descriptors and prefix arrays.
static size_t layout_batch(const BatchPlan& b, void* ws, std::vector<SetDev>* descs, std::vector<int64_t>* prefix,
                           unsigned long long** counters, SetDev** dev_sets, int64_t** dev_prefix) {
  Carver c(ws, ~size_t(0));
  const int ns = int(b.sets.size());
  unsigned long long* cnt = c.take<unsigned long long>(kCounters);
  SetDev* ds = c.take<SetDev>(ns);
  int64_t* dp = c.take<int64_t>(size_t(PF_COUNT) * (ns + 1));
  if (descs) descs->assign(ns, SetDev{});
  if (prefix) prefix->assign(size_t(PF_COUNT) * (ns + 1), 0);
  int64_t acc[PF_COUNT] = {0};
  const size_t es = elem_size(b.prec);
  for (int r = 0; r < ns; ++r) {
    const kde_batch_set& in = b.sets[b.order[r]];
    SetDev d{};
    d.n = in.N;
    d.n_cv = in.n_cv ? in.n_cv : in.N;
    d.x = in.x;
    d.L = in.L;
    d.M = in.M;
    const SortPlan sp = make_sort_plan(d.n_cv);
    d.cells = sp.cells;
    d.chunk = deposit_chunk(in.N);
    const int64_t ntiles = ceil_div(d.n_cv, kCvTile);
    d.units = ntiles * (ntiles + 1) / 2;
    d.g_cv = ceil_div(d.units, kSumRows);
    d.chunks = ceil_div(in.N, d.chunk);
    d.g_dep = ceil_div(d.chunks, kSumRows);
    d.blocks = ceil_div(in.N, kBlock);
    d.g_ad = ceil_div(d.blocks, kSumRows);
    d.packed = b.prec == KDE_F64 ? static_cast<void*>(c.take<double>(2 * size_t(d.n_cv)))
                                 : static_cast<void*>(c.take<uint32_t>(size_t(d.n_cv)));
    d.partials = c.take<double>(size_t(d.units) * 2 * b.B);
    d.cv_l1 = c.take<double>(size_t(d.g_cv) * 2 * b.B);
    d.dep_part = c.take<double>(size_t(d.chunks) * in.M);
    d.dep_l1 = c.take<double>(size_t(d.g_dep) * in.M);
    d.pilot = in.pilot ? in.pilot : c.take<double>(size_t(in.M));
    d.ad_part = c.take<double>(size_t(d.blocks) * 2);
    d.ad_l1 = c.take<double>(size_t(d.g_ad) * 2);
    d.ad_sums = c.take<double>(2);
    d.kappa_i = in.kappa_i ? in.kappa_i : static_cast<void*>(c.take<char>(size_t(in.N) * es));
    d.rho = in.rho;
    d.cv = in.cv;
    d.kstar = c.take<double>(1);
    d.kstar_user = in.kappa_star;
    if (descs) (*descs)[r] = d;
    const int64_t per[PF_COUNT] = {d.units, d.g_cv, d.chunks, d.g_dep, d.blocks, d.g_ad};
    for (int k = 0; k < PF_COUNT; ++k) {
      if (prefix) (*prefix)[size_t(k) * (ns + 1) + r] = acc[k];
      acc[k] += per[k];
    }
  }
  for (int k = 0; k < PF_COUNT; ++k)
    if (prefix) (*prefix)[size_t(k) * (ns + 1) + ns] = acc[k];
  if (counters) *counters = cnt;
  if (dev_sets) *dev_sets = ds;
  if (dev_prefix) *dev_prefix = dp;
  return c.used;
}

// Workgroups to launch for a persistent phase kernel: what the device keeps
// resident, but no more than the phase has units.
template <typename K>
static unsigned persistent_grid(K kernel, size_t dyn_lds, int64_t units) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, dyn_lds) != hipSuccess || per < 1) per = 1;
  int64_t g = int64_t(cus) * per;
  if (units < g) g = units;
  return unsigned(g < 1 ? 1 : g);
}

template <typename T, int G>
static kde_status enqueue_batch(const BatchPlan& b, const BatchArgs& a, const std::vector<int64_t>& prefix, hipStream_t s) {
  const int ns = int(b.sets.size());
  auto total = [&](int pf) { return prefix[size_t(pf) * (ns + 1) + ns]; };
  const CvConsts<T> K = make_consts<T>(b.kappas.data(), b.B);
  KappaList kl{};
  for (int k = 0; k < b.B; ++k) kl.k[k] = b.kappas[k];
  const size_t dep_lds = 2 * size_t(b.max_M) * sizeof(T);
  const size_t pack_lds = size_t(b.max_cells) * sizeof(int);

  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(kBlock), 0, s, a.counters);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_pack_kernel<T>, dim3(persistent_grid(batch_pack_kernel<T>, pack_lds, ns)), dim3(kBlock),
                     pack_lds, s, a);
  KDE_CHECK_LAUNCH();
  for (size_t k = 0; k < b.bucket_bc.size(); ++k) {
    const int64_t lo = prefix[size_t(PF_PAIRS) * (ns + 1) + b.bucket_begin[k]];
    const int64_t hi = prefix[size_t(PF_PAIRS) * (ns + 1) + b.bucket_begin[k + 1]];
    const int ph = int(PH_COUNT + k);
    switch (b.bucket_bc[k]) {
      case 4:
        hipLaunchKernelGGL((batch_pairs_kernel<T, 4>), dim3(persistent_grid(batch_pairs_kernel<T, 4>, 0, hi - lo)),
                           dim3(kBlock), 0, s, a, K, ph, lo, hi);
        break;
      case 8:
        hipLaunchKernelGGL((batch_pairs_kernel<T, 8>), dim3(persistent_grid(batch_pairs_kernel<T, 8>, 0, hi - lo)),
                           dim3(kBlock), 0, s, a, K, ph, lo, hi);
        break;
      default:
        hipLaunchKernelGGL((batch_pairs_kernel<T, 16>), dim3(persistent_grid(batch_pairs_kernel<T, 16>, 0, hi - lo)),
                           dim3(kBlock), 0, s, a, K, ph, lo, hi);
        break;
    }
    KDE_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(batch_level1_kernel<SRC_CV>,
                     dim3(persistent_grid(batch_level1_kernel<SRC_CV>, 0, total(PF_CV_L1))), dim3(kBlock), 0, s, a,
                     int(PH_CV_L1), int(PF_CV_L1));
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_cv_finalize_kernel, dim3(persistent_grid(batch_cv_finalize_kernel, 0, ns)), dim3(kBlock), 0,
                     s, a, kl);
  KDE_CHECK_LAUNCH();
  for (int pass = 0; pass < 2; ++pass) {
    const bool adaptive = pass == 1;
    if (adaptive) {
      hipLaunchKernelGGL(batch_adapt_log_kernel<T>,
                         dim3(persistent_grid(batch_adapt_log_kernel<T>, 0, total(PF_BLOCKS))), dim3(kBlock), 0, s, a);
      KDE_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_level1_kernel<SRC_AD>,
                         dim3(persistent_grid(batch_level1_kernel<SRC_AD>, 0, total(PF_AD_L1))), dim3(kBlock), 0, s,
                         a, int(PH_AD_L1), int(PF_AD_L1));
      KDE_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_level2_kernel<1>, dim3(persistent_grid(batch_level2_kernel<1>, 0, ns)), dim3(kBlock), 0,
                         s, a, int(PH_AD_L2));
      KDE_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_adapt_apply_kernel<T>,
                         dim3(persistent_grid(batch_adapt_apply_kernel<T>, 0, total(PF_BLOCKS))), dim3(kBlock), 0, s,
                         a);
      KDE_CHECK_LAUNCH();
    }
    {
      if (adaptive)
        hipLaunchKernelGGL((batch_deposit_kernel<T, true, G>),
                           dim3(persistent_grid(batch_deposit_kernel<T, true, G>, dep_lds, total(PF_CHUNKS))),
                           dim3(kBlock), dep_lds, s, a, int(PH_RHO_DEP));
      else
        hipLaunchKernelGGL((batch_deposit_kernel<T, false, G>),
                           dim3(persistent_grid(batch_deposit_kernel<T, false, G>, dep_lds, total(PF_CHUNKS))),
                           dim3(kBlock), dep_lds, s, a, int(PH_PIL_DEP));
    }
    KDE_CHECK_LAUNCH();
    hipLaunchKernelGGL(batch_level1_kernel<SRC_DEP>,
                       dim3(persistent_grid(batch_level1_kernel<SRC_DEP>, 0, total(PF_DEP_L1))), dim3(kBlock), 0, s, a,
                       int(adaptive ? PH_RHO_L1 : PH_PIL_L1), int(PF_DEP_L1));
    KDE_CHECK_LAUNCH();
    if (adaptive)
      hipLaunchKernelGGL(batch_level2_kernel<2>, dim3(persistent_grid(batch_level2_kernel<2>, 0, ns)), dim3(kBlock), 0,
                         s, a, int(PH_RHO_L2));
    else
      hipLaunchKernelGGL(batch_level2_kernel<0>, dim3(persistent_grid(batch_level2_kernel<0>, 0, ns)), dim3(kBlock), 0,
                         s, a, int(PH_PIL_L2));
    KDE_CHECK_LAUNCH();
  }
  return KDE_OK;
}

template <typename T>
static kde_status enqueue_batch_t(const BatchPlan& b, const BatchArgs& a, const std::vector<int64_t>& pf, hipStream_t s) {
  const int g = int(ceil_div(b.max_M, kBlock));
  if (g <= 1) return enqueue_batch<T, 1>(b, a, pf, s);
  if (g <= 2) return enqueue_batch<T, 2>(b, a, pf, s);
  if (g <= 4) return enqueue_batch<T, 4>(b, a, pf, s);
  if (g <= 8) return enqueue_batch<T, 8>(b, a, pf, s);
  return enqueue_batch<T, 16>(b, a, pf, s);
}

// Descriptors of the plan written into `ws` (host images).
static void batch_images(const BatchPlan& b, void* ws, std::vector<SetDev>& descs, std::vector<int64_t>& prefix,
                         BatchArgs& a) {
  unsigned long long* counters = nullptr;
  SetDev* dsets = nullptr;
  int64_t* dpref = nullptr;
  layout_batch(b, ws, &descs, &prefix, &counters, &dsets, &dpref);
  a = BatchArgs{dsets, dpref, counters, int(b.sets.size()), b.B, b.alpha};
}

kde_status batch_plan_make(const kde_batch_set* sets_h, int nsets, int prec, int B, const double* kappas_h,
                           double alpha, BatchPlan& im) {
  if (!sets_h || nsets < 1) return fail(KDE_E_INVALID_ARG, "need at least one set");
  if (prec != KDE_F64 && prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32");
  if (B < 1 || B > KDE_MAX_KAPPAS || !kappas_h) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d]", KDE_MAX_KAPPAS);
  for (int k = 0; k < B; ++k) {
    if (!std::isfinite(kappas_h[k]) || kappas_h[k] < 0.0) return fail(KDE_E_INVALID_ARG, "kappa %d must be finite and >= 0", k);
    if (k > 0 && !(kappas_h[k] > kappas_h[k - 1])) return fail(KDE_E_INVALID_ARG, "kappas must be strictly ascending");
  }
  if (!std::isfinite(alpha) || alpha < 0.0) return fail(KDE_E_INVALID_ARG, "alpha must be finite and >= 0");
  im = BatchPlan{};
  for (int s = 0; s < nsets; ++s) {
    const kde_batch_set& in = sets_h[s];
    if (in.N < 2 || in.N > kMaxN) return fail(KDE_E_INVALID_ARG, "set %d: N must lie in [2, %lld]", s, (long long)kMaxN);
    if (!in.x || !in.rho) return fail(KDE_E_INVALID_ARG, "set %d: x and rho must not be NULL", s);
    if (in.n_cv != 0 && (in.n_cv < 2 || in.n_cv > in.N))
      return fail(KDE_E_INVALID_ARG, "set %d: n_cv must be 0 or lie in [2, N]", s);
    if (!std::isfinite(in.L) || !(in.L > 0.0)) return fail(KDE_E_INVALID_ARG, "set %d: L must be finite and > 0", s);
    if (in.M < 2 || in.M > kMaxM) return fail(KDE_E_INVALID_ARG, "set %d: M must lie in [2, %d]", s, kMaxM);
    im.max_M = std::max(im.max_M, int(in.M));
    im.max_n = std::max(im.max_n, in.N);
    im.max_cells = std::max(im.max_cells, make_sort_plan(in.n_cv ? in.n_cv : in.N).cells);
  }
  im.prec = prec;
  im.B = B;
  im.alpha = alpha;
  im.kappas.assign(kappas_h, kappas_h + B);
  im.sets.assign(sets_h, sets_h + nsets);
  im.order.resize(nsets);
  std::iota(im.order.begin(), im.order.end(), 0);
  // largest pair-sum work first (stable, so equal sets keep caller order)
  auto ncv = [&](int i) { return im.sets[i].n_cv ? im.sets[i].n_cv : im.sets[i].N; };
  std::stable_sort(im.order.begin(), im.order.end(), [&](int a, int c) { return ncv(a) > ncv(c); });
  // contiguous runs of equal tuned pass size along the LPT order (at most
  // one per entry of the tuning table, as N decreases along the order)
  for (int r = 0; r < nsets; ++r) {
    const int bc = tuned_chunk(prec, ncv(im.order[r]));
    if (im.bucket_bc.empty() || im.bucket_bc.back() != bc) {
      if (int(im.bucket_bc.size()) == kMaxBuckets) return fail(KDE_E_INTERNAL, "too many pass-size buckets");
      im.bucket_begin.push_back(r);
      im.bucket_bc.push_back(bc);
    }
  }
  im.bucket_begin.push_back(nsets);
  im.ws_need = layout_batch(im, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  return KDE_OK;
}

size_t batch_staging_bytes(const BatchPlan& b) {
  const size_t ns = b.sets.size();
  return ns * sizeof(SetDev) + size_t(PF_COUNT) * (ns + 1) * sizeof(int64_t) + 64;
}

kde_status batch_plan_enqueue(const BatchPlan& b, void* ws, hipStream_t s, void* staging_h) {
  std::vector<SetDev> descs;
  std::vector<int64_t> prefix;
  BatchArgs a{};
  batch_images(b, ws, descs, prefix, a);
  const size_t db = descs.size() * sizeof(SetDev), pb = prefix.size() * sizeof(int64_t);
  char* st = static_cast<char*>(staging_h);
  memcpy(st, descs.data(), db);
  memcpy(st + db, prefix.data(), pb);
  KDE_TRY_HIP(hipMemcpyAsync(const_cast<SetDev*>(a.sets), st, db, hipMemcpyHostToDevice, s));
  KDE_TRY_HIP(hipMemcpyAsync(const_cast<int64_t*>(a.prefix), st + db, pb, hipMemcpyHostToDevice, s));
  return b.prec == KDE_F64 ? enqueue_batch_t<double>(b, a, prefix, s) : enqueue_batch_t<float>(b, a, prefix, s);
}

// Upload descriptors and capture the graph for workspace `ws`.
static kde_status build_graph(kde_batch_graph& g, const BatchPlan& b, void* ws, size_t ws_bytes) {
  std::vector<SetDev> descs;
  std::vector<int64_t> prefix;
  BatchArgs a{};
  batch_images(b, ws, descs, prefix, a);
  KDE_TRY_HIP(hipMemcpy(const_cast<SetDev*>(a.sets), descs.data(), descs.size() * sizeof(SetDev), hipMemcpyHostToDevice));
  KDE_TRY_HIP(hipMemcpy(const_cast<int64_t*>(a.prefix), prefix.data(), prefix.size() * sizeof(int64_t),
                        hipMemcpyHostToDevice));
  g.reset();
  KDE_TRY_HIP(hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
  KDE_TRY_HIP(hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal));
  kde_status st = b.prec == KDE_F64 ? enqueue_batch_t<double>(b, a, prefix, g.cap)
                                    : enqueue_batch_t<float>(b, a, prefix, g.cap);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(g.cap, &graph);
  if (st != KDE_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(KDE_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
  g.graph = graph;
  KDE_TRY_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  g.ws = ws;
  g.ws_bytes = ws_bytes;
  return KDE_OK;
}

}  // namespace kde

using namespace kde;

struct kde_batch {
  BatchPlan plan;
  kde_batch_graph graph;
};

extern "C" {

kde_status kde_batch_plan(const kde_batch_set* sets_h, int32_t nsets, int32_t prec, int32_t B,
                          const double* kappas_h, double alpha, kde_batch** out_h) {
  clear_error();
  if (!out_h) return fail(KDE_E_INVALID_ARG, "out_h is NULL");
  *out_h = nullptr;
  std::unique_ptr<kde_batch> b(new kde_batch());
  KDE_RETURN_IF(batch_plan_make(sets_h, nsets, prec, B, kappas_h, alpha, b->plan));
  *out_h = b.release();
  return KDE_OK;
}

kde_status kde_batch_workspace_size(const kde_batch* b, size_t* bytes_h) {
  clear_error();
  if (!b || !bytes_h) return fail(KDE_E_INVALID_ARG, "batch and bytes_h must not be NULL");
  *bytes_h = b->plan.ws_need;
  return KDE_OK;
}

kde_status kde_batch_run(kde_batch* b, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!b) return fail(KDE_E_NOT_FOUND, "batch is NULL");
  const BatchPlan& im = b->plan;
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, im.ws_need));
  KDE_RETURN_IF(check_lds(2 * size_t(im.max_M) * elem_size(im.prec) + kDepMaxChunk * 32 + kBlock * 8));
  if (!b->graph.exec || b->graph.ws != ws || b->graph.ws_bytes != ws_bytes)
    KDE_RETURN_IF(build_graph(b->graph, im, ws, ws_bytes));
  KDE_TRY_HIP(hipGraphLaunch(b->graph.exec, static_cast<hipStream_t>(stream)));
  return KDE_OK;
}

kde_status kde_batch_destroy(kde_batch* b) {
  clear_error();
  delete b;
  return KDE_OK;
}

}  // extern "C"
