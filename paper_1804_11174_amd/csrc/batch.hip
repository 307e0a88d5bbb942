// Batching form: many independent particle sets through the whole plain
// path (CV scan over a shared list of concentrations, pilot deposit at each
// set's kappa*, adaptive widths, adaptive deposit) in one hipGraph launch.
//
// The graph holds one kernel per phase over the work units of every set
// -- (set), (set, sort block), (set, pair slot, concentration group),
// (set, particle chunk) or (set, row block) -- with the sets ordered by
// decreasing CV cost so that the long pair-sum work starts first. The pair
// phase runs one workgroup per unit; the light phases run about as many
// workgroups as the device keeps resident, pulling units from the phase's
// own device counter. Phases follow each other in the graph, so no
// workgroup ever waits on another. Every unit runs the same device code as
// the one-set entry points and writes its own slot, and every reduction has
// the one-set entry points' fixed order, so each set's results are bitwise
// identical to running it alone.
#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "batch_internal.hpp"
#include "dev_cv.hpp"
#include "dev_density.hpp"
#include "dev_layout.hpp"
#include "dev_reduce.hpp"

namespace kde {

// Work counters of the phases that claim units (zeroed by the first kernel
// of every launch).
enum Phase {
  PH_SORT_HIST, PH_SORT_SCAN, PH_SORT_SCATTER, PH_CV_L1, PH_CV_FIN, PH_PIL_L1, PH_PIL_L2, PH_AD_LOG, PH_AD_L1,
  PH_AD_L2, PH_AD_APPLY, PH_RHO_L1, PH_RHO_L2, PH_COUNT
};
// The pair phase runs once per pass-size bucket, one workgroup per unit.
constexpr int kMaxBuckets = 64;
constexpr int kCounters = PH_COUNT;

// Per-set description as the kernels see it (lives in the workspace).
struct SetDev {
  int64_t n;
  int64_t n_cv;  // particles the CV scan uses (a prefix)
  const void* x;
  double L;
  int M, cells, chunk, sblocks;  // sblocks: blocks of the cell sort
  int gsize, groups;              // pair units: concentrations per unit, units per slot
  int64_t schunk;                 // particles per sort block
  int64_t slots, g_cv, chunks, g_dep, blocks, g_ad;  // slots: rows of CV partial sums (cv_slots)
  int32_t* hist;      // cells x sblocks, cell-major
  void* packed;
  double* partials;   // slots x 2B
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
  uint32_t* status;   // the set's numeric status word (KDE_NUMERIC_* bits)
};

// Unit prefix sums, one array of nsets + 1 per multi-unit phase.
enum Prefix { PF_PAIRS, PF_CV_L1, PF_CHUNKS, PF_DEP_L1, PF_BLOCKS, PF_AD_L1, PF_SORT, PF_COUNT };

struct BatchArgs {
  const SetDev* sets;
  const int64_t* prefix;  // PF_COUNT x (nsets + 1)
  unsigned long long* counters;
  uint32_t* statuses;     // nsets numeric status words, in the caller's set order
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

// Values known to be equal in every lane, moved to scalar registers (the
// compiler cannot prove a loaded set descriptor uniform by itself).
__device__ __forceinline__ int uni32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}
template <typename P>
__device__ __forceinline__ P* uni_ptr(P* p) {
  return reinterpret_cast<P*>(uni64(reinterpret_cast<int64_t>(p)));
}

// Claim the next unit of a phase for the whole workgroup. The value is
// the same in every lane; reading it through readfirstlane lets the
// compiler know that, so the unit's set descriptor and loop bounds live in
// scalar registers.
__device__ __forceinline__ int64_t claim(unsigned long long* counter, int64_t* slot) {
  if (threadIdx.x == 0) *slot = int64_t(atomicAdd(counter, 1ull));
  __syncthreads();
  const int64_t v = *slot;
  __syncthreads();
  return uni64(v);
}

__global__ void __launch_bounds__(kBlock) batch_zero_kernel(unsigned long long* counters, uint32_t* statuses,
                                                            int nsets) {
  if (threadIdx.x < kCounters) counters[threadIdx.x] = 0ull;
  for (int k = threadIdx.x; k < nsets; k += kBlock) statuses[k] = 0u;
}

// The stable cell sort of every set's CV prefix in three phases, with the
// one-set path's block decomposition: per-block histograms, one scan per
// set, per-block scatters.
template <typename T>
__global__ void __launch_bounds__(kBlock) batch_sort_hist_kernel(BatchArgs a) {
  __shared__ int64_t slot;
  extern __shared__ int lh[];
  const int64_t* pf = a.prefix + PF_SORT * (a.nsets + 1);
  const int64_t total = pf[a.nsets];
  for (;;) {
    const int64_t u = claim(&a.counters[PH_SORT_HIST], &slot);
    if (u >= total) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int b = int(u - pf[si]);
    const int64_t lo = int64_t(b) * s.schunk;
    sort_hist_block<T>(static_cast<const T*>(s.x), lo, min(s.n_cv, lo + s.schunk), s.L, s.cells, b, s.sblocks, lh,
                       s.hist, s.status);
  }
}

__global__ void __launch_bounds__(kBlock) batch_sort_scan_kernel(BatchArgs a) {
  __shared__ int64_t slot;
  __shared__ int tot[kBlock / 64];
  for (;;) {
    const int64_t u = claim(&a.counters[PH_SORT_SCAN], &slot);
    if (u >= a.nsets) break;
    const SetDev& s = a.sets[u];
    block_scan_global(s.hist, int64_t(s.cells) * s.sblocks, tot);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) batch_sort_scatter_kernel(BatchArgs a) {
  using P = typename Packed<T>::type;
  __shared__ int64_t slot;
  extern __shared__ int base[];
  const int64_t* pf = a.prefix + PF_SORT * (a.nsets + 1);
  const int64_t total = pf[a.nsets];
  for (;;) {
    const int64_t u = claim(&a.counters[PH_SORT_SCATTER], &slot);
    if (u >= total) break;
    const int si = find_set(pf, a.nsets, u);
    const SetDev& s = a.sets[si];
    const int b = int(u - pf[si]);
    const int64_t lo = int64_t(b) * s.schunk;
    sort_scatter_block<T, P>(static_cast<const T*>(s.x), lo, min(s.n_cv, lo + s.schunk), s.L, s.cells, b, s.sblocks,
                             s.hist, base, static_cast<P*>(s.packed), nullptr);
  }
}

// Pair units [u_lo, u_hi) of the flattened list (one pass-size bucket), a
// unit being a (set, slot, concentration group), one workgroup per unit. The list follows the cost order of the sets, and
// workgroups are dispatched in index order, so the largest sets start
// first without a work counter; a loop over claimed units would keep more
// registers live and lower the occupancy of this, the heaviest phase.
template <typename T, int BC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PairWaves<T, BC>::value))) batch_pairs_kernel(BatchArgs a, CvConsts<T> K, int64_t u_lo, int64_t u_hi) {
  using P = typename Packed<T>::type;
  __shared__ CvSmem<T, BC> sm;
  const int64_t* pf = a.prefix + PF_PAIRS * (a.nsets + 1);
  {
    const int64_t u = u_lo + int64_t(blockIdx.x);
    if (u >= u_hi) return;
    const int si = uni32(find_set(pf, a.nsets, u));
    const SetDev& s = a.sets[si];
    const int64_t q = u - uni64(pf[si]);
    const int groups = uni32(s.groups), gsize = uni32(s.gsize);
    const int64_t r = q / groups;
    const int b_lo = int(q - r * groups) * gsize;
    cv_slot<T, BC>(uni_ptr(static_cast<const P*>(s.packed)), uni64(s.n_cv), uni32(s.cells), s.L, r, uni64(s.slots),
                   K, b_lo, min(K.B, b_lo + gsize), uni_ptr(s.partials) + r * 2 * K.B, sm);
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
      in = s.partials; l1 = s.cv_l1; rows = s.slots; cols = 2 * a.B;
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
__global__ void __launch_bounds__(kBlock) batch_deposit_kernel(BatchArgs a) {
  __shared__ DepSmem<T> sm;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int64_t* pf = a.prefix + PF_CHUNKS * (a.nsets + 1);
  SinCos<T>* tab = reinterpret_cast<SinCos<T>*>(dyn);
  const int64_t u = int64_t(blockIdx.x);
  if (u >= pf[a.nsets]) return;
  const int si = uni32(find_set(pf, a.nsets, u));
  const SetDev& s = a.sets[si];
  const int64_t c = u - uni64(pf[si]);
  const int M = uni32(s.M);
  const int chunk = uni32(s.chunk);
  node_table(M, tab);
  const int64_t lo = c * chunk;
  const int cnt = int(min(int64_t(chunk), uni64(s.n) - lo));
  deposit_block<T, PER, G>(uni_ptr(static_cast<const T*>(s.x)), uni_ptr(static_cast<const T*>(s.kappa_i)),
                           PER ? 0.0 : *s.kstar, M, s.L, lo, cnt, uni_ptr(s.dep_part) + c * M, tab, sm,
                           uni_ptr(s.status));
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
    adapt_logsum_block<T>(static_cast<const T*>(s.x), s.n, s.M, s.L, s.pilot, b, s.ad_part + 2 * b, r0, r1,
                          s.status);
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
                           unsigned long long** counters, SetDev** dev_sets, int64_t** dev_prefix,
                           uint32_t** statuses_out = nullptr) {
  Carver c(ws, ~size_t(0));
  const int ns = int(b.sets.size());
  unsigned long long* cnt = c.take<unsigned long long>(kCounters);
  uint32_t* statuses = c.take<uint32_t>(size_t(ns));
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
    d.sblocks = sp.blocks;
    d.schunk = sp.chunk;
    d.chunk = deposit_chunk(in.N);
    d.slots = cv_slots(d.n_cv);
    const PairTuning tp = tuned_pass(b.prec, d.n_cv);
    d.gsize = pair_group_size(tp, b.B);
    d.groups = pair_groups(tp, b.B);
    d.g_cv = ceil_div(d.slots, kSumRows);
    d.chunks = ceil_div(in.N, d.chunk);
    d.g_dep = ceil_div(d.chunks, kSumRows);
    d.blocks = ceil_div(in.N, kBlock);
    d.g_ad = ceil_div(d.blocks, kSumRows);
    d.hist = c.take<int32_t>(size_t(d.cells) * size_t(d.sblocks));
    d.packed = b.prec == KDE_F64 ? static_cast<void*>(c.take<double>(Packed<double>::per_particle * size_t(d.n_cv)))
                                 : static_cast<void*>(c.take<uint32_t>(size_t(d.n_cv)));
    d.partials = c.take<double>(size_t(d.slots) * 2 * b.B);
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
    d.status = statuses + b.order[r];
    if (descs) (*descs)[r] = d;
    const int64_t per[PF_COUNT] = {d.slots * d.groups, d.g_cv, d.chunks, d.g_dep, d.blocks, d.g_ad, int64_t(d.sblocks)};
    for (int k = 0; k < PF_COUNT; ++k) {
      if (prefix) (*prefix)[size_t(k) * (ns + 1) + r] = acc[k];
      acc[k] += per[k];
    }
  }
  for (int k = 0; k < PF_COUNT; ++k)
    if (prefix) (*prefix)[size_t(k) * (ns + 1) + ns] = acc[k];
  if (counters) *counters = cnt;
  if (statuses_out) *statuses_out = statuses;
  if (dev_sets) *dev_sets = ds;
  if (dev_prefix) *dev_prefix = dp;
  return c.used;
}

// Workgroups to launch for a phase kernel: with resident grids what the
// device keeps resident, but no more than the phase has units; otherwise
// one per unit. The occupancy of each (kernel, LDS, device) is queried
// once.
static int resident_blocks(const void* kernel, size_t dyn_lds, int dev) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int> cache;
  const auto key = std::make_tuple(kernel, dyn_lds, dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, dyn_lds) != hipSuccess || per < 1) per = 1;
  return cache[key] = cus * per;
}

template <typename K>
static unsigned launch_grid(const BatchPlan& b, K kernel, size_t dyn_lds, int64_t units) {
  int64_t g = int64_t(1) << 30;
  if (b.resident_grids) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    g = resident_blocks(reinterpret_cast<const void*>(kernel), dyn_lds, dev);
  }
  if (units < g) g = units;
  return unsigned(g < 1 ? 1 : g);
}

template <typename T, int G>
static kde_status enqueue_batch(const BatchPlan& b, const BatchArgs& a, const std::vector<int64_t>& prefix, hipStream_t s) {
  const int ns = int(b.sets.size());
  auto total = [&](int pf) { return prefix[size_t(pf) * (ns + 1) + ns]; };
  const CvConsts<T> K = make_consts<T>(b.kappas.data(), b.B);
  const KappaList kl = make_kappa_list<T>(b.kappas.data(), b.B);
  const size_t dep_lds = 2 * size_t(b.max_M) * sizeof(T);
  const size_t pack_lds = size_t(b.max_cells) * sizeof(int);

  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(kBlock), 0, s, a.counters, a.statuses, ns);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_sort_hist_kernel<T>, dim3(launch_grid(b, batch_sort_hist_kernel<T>, pack_lds, total(PF_SORT))),
                     dim3(kBlock), pack_lds, s, a);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_sort_scan_kernel, dim3(launch_grid(b, batch_sort_scan_kernel, 0, ns)), dim3(kBlock), 0, s, a);
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_sort_scatter_kernel<T>,
                     dim3(launch_grid(b, batch_sort_scatter_kernel<T>, pack_lds, total(PF_SORT))), dim3(kBlock),
                     pack_lds, s, a);
  KDE_CHECK_LAUNCH();
  for (size_t k = 0; k < b.bucket_bc.size(); ++k) {
    const int64_t lo = prefix[size_t(PF_PAIRS) * (ns + 1) + b.bucket_begin[k]];
    const int64_t hi = prefix[size_t(PF_PAIRS) * (ns + 1) + b.bucket_begin[k + 1]];
    if (hi - lo > int64_t(0x7fffffff)) return fail(KDE_E_INVALID_ARG, "too many pair units for one launch");
    const dim3 grid{unsigned(hi - lo)};
    with_pass_size<T>(b.bucket_bc[k], [&](auto bc) {
      hipLaunchKernelGGL((batch_pairs_kernel<T, decltype(bc)::value>), grid, dim3(kBlock), 0, s, a, K, lo, hi);
    });
    KDE_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(batch_level1_kernel<SRC_CV>,
                     dim3(launch_grid(b, batch_level1_kernel<SRC_CV>, 0, total(PF_CV_L1))), dim3(kBlock), 0, s, a,
                     int(PH_CV_L1), int(PF_CV_L1));
  KDE_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_cv_finalize_kernel, dim3(launch_grid(b, batch_cv_finalize_kernel, 0, ns)), dim3(kBlock), 0,
                     s, a, kl);
  KDE_CHECK_LAUNCH();
  for (int pass = 0; pass < 2; ++pass) {
    const bool adaptive = pass == 1;
    if (adaptive) {
      hipLaunchKernelGGL(batch_adapt_log_kernel<T>,
                         dim3(launch_grid(b, batch_adapt_log_kernel<T>, 0, total(PF_BLOCKS))), dim3(kBlock), 0, s, a);
      KDE_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_level1_kernel<SRC_AD>,
                         dim3(launch_grid(b, batch_level1_kernel<SRC_AD>, 0, total(PF_AD_L1))), dim3(kBlock), 0, s,
                         a, int(PH_AD_L1), int(PF_AD_L1));
      KDE_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_level2_kernel<1>, dim3(launch_grid(b, batch_level2_kernel<1>, 0, ns)), dim3(kBlock), 0,
                         s, a, int(PH_AD_L2));
      KDE_CHECK_LAUNCH();
      hipLaunchKernelGGL(batch_adapt_apply_kernel<T>,
                         dim3(launch_grid(b, batch_adapt_apply_kernel<T>, 0, total(PF_BLOCKS))), dim3(kBlock), 0, s,
                         a);
      KDE_CHECK_LAUNCH();
    }
    {
      if (adaptive)
        hipLaunchKernelGGL((batch_deposit_kernel<T, true, G>), dim3(unsigned(total(PF_CHUNKS))), dim3(kBlock),
                           dep_lds, s, a);
      else
        hipLaunchKernelGGL((batch_deposit_kernel<T, false, G>), dim3(unsigned(total(PF_CHUNKS))), dim3(kBlock),
                           dep_lds, s, a);
    }
    KDE_CHECK_LAUNCH();
    hipLaunchKernelGGL(batch_level1_kernel<SRC_DEP>,
                       dim3(launch_grid(b, batch_level1_kernel<SRC_DEP>, 0, total(PF_DEP_L1))), dim3(kBlock), 0, s, a,
                       int(adaptive ? PH_RHO_L1 : PH_PIL_L1), int(PF_DEP_L1));
    KDE_CHECK_LAUNCH();
    if (adaptive)
      hipLaunchKernelGGL(batch_level2_kernel<2>, dim3(launch_grid(b, batch_level2_kernel<2>, 0, ns)), dim3(kBlock), 0,
                         s, a, int(PH_RHO_L2));
    else
      hipLaunchKernelGGL(batch_level2_kernel<0>, dim3(launch_grid(b, batch_level2_kernel<0>, 0, ns)), dim3(kBlock), 0,
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
  uint32_t* statuses = nullptr;
  layout_batch(b, ws, &descs, &prefix, &counters, &dsets, &dpref, &statuses);
  a = BatchArgs{dsets, dpref, counters, statuses, int(b.sets.size()), b.B, b.alpha};
}

kde_status batch_plan_make(const kde_batch_set* sets_h, int nsets, int prec, int B, const double* kappas_h,
                           double alpha, BatchPlan& im) {
  if (!sets_h || nsets < 1) return fail(KDE_E_INVALID_ARG, "need at least one set");
  if (prec != KDE_F64 && prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32");
  if (B < 1 || B > KDE_MAX_KAPPAS || !kappas_h) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d]", KDE_MAX_KAPPAS);
  for (int k = 0; k < B; ++k) {
    if (!std::isfinite(kappas_h[k]) || kappas_h[k] < 0.0 || kappas_h[k] > KDE_MAX_CV_KAPPA)
      return fail(KDE_E_INVALID_ARG, "kappa %d must lie in [0, %g]", k, KDE_MAX_CV_KAPPA);
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
    const int bc = tuned_pass(prec, ncv(im.order[r])).chunk;
    if (im.bucket_bc.empty() || im.bucket_bc.back() != bc) {
      if (int(im.bucket_bc.size()) == kMaxBuckets) return fail(KDE_E_INTERNAL, "too many pass-size buckets");
      im.bucket_begin.push_back(r);
      im.bucket_bc.push_back(bc);
    }
  }
  im.bucket_begin.push_back(nsets);
  for (size_t k = 0; k + 1 < im.bucket_begin.size(); ++k) {
    int64_t units = 0;
    for (int r = im.bucket_begin[k]; r < im.bucket_begin[k + 1]; ++r) {
      units += cv_slots(ncv(im.order[r])) * pair_groups(tuned_pass(prec, ncv(im.order[r])), B);
      if (units > int64_t(0x7fffffff)) return fail(KDE_E_INVALID_ARG, "too many CV pair units for one launch");
    }
  }
  im.ws_need = layout_batch(im, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  return KDE_OK;
}

static size_t staged_status_offset(const BatchPlan& b) {
  const size_t ns = b.sets.size();
  return round_up(ns * sizeof(SetDev) + size_t(PF_COUNT) * (ns + 1) * sizeof(int64_t), 64);
}

size_t batch_staging_bytes(const BatchPlan& b) {
  return staged_status_offset(b) + b.sets.size() * sizeof(uint32_t) + 64;
}

const uint32_t* batch_staged_status(const BatchPlan& b, const void* staging_h) {
  return reinterpret_cast<const uint32_t*>(static_cast<const char*>(staging_h) + staged_status_offset(b));
}

uint32_t* batch_status_words(const BatchPlan& b, void* ws) {
  uint32_t* st = nullptr;
  layout_batch(b, ws, nullptr, nullptr, nullptr, nullptr, nullptr, &st);
  return st;
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
  KDE_RETURN_IF(b.prec == KDE_F64 ? enqueue_batch_t<double>(b, a, prefix, s) : enqueue_batch_t<float>(b, a, prefix, s));
  KDE_TRY_HIP(hipMemcpyAsync(st + staged_status_offset(b), a.statuses, b.sets.size() * sizeof(uint32_t),
                             hipMemcpyDeviceToHost, s));
  return KDE_OK;
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
  KDE_RETURN_IF(check_lds(2 * size_t(im.max_M) * elem_size(im.prec) +
                          (im.prec == KDE_F64 ? sizeof(DepSmem<double>) : sizeof(DepSmem<float>))));
  if (!b->graph.exec || b->graph.ws != ws || b->graph.ws_bytes != ws_bytes)
    KDE_RETURN_IF(build_graph(b->graph, im, ws, ws_bytes));
  KDE_TRY_HIP(hipGraphLaunch(b->graph.exec, static_cast<hipStream_t>(stream)));
  return KDE_OK;
}

kde_status kde_batch_status(kde_batch* b, uint32_t* flags_h, void* stream) {
  clear_error();
  if (!b || !flags_h) return fail(KDE_E_INVALID_ARG, "batch and flags_h must not be NULL");
  if (!b->graph.exec) return fail(KDE_E_INVALID_ARG, "the batch has not been run");
  KDE_TRY_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  const size_t ns = b->plan.sets.size();
  KDE_TRY_HIP(hipMemcpy(flags_h, batch_status_words(b->plan, b->graph.ws), ns * sizeof(uint32_t),
                        hipMemcpyDeviceToHost));
  for (size_t k = 0; k < ns; ++k)
    if (flags_h[k]) return fail(KDE_E_NUMERIC, "set %zu met non-finite values (flags %u)", k, flags_h[k]);
  return KDE_OK;
}

kde_status kde_batch_destroy(kde_batch* b) {
  clear_error();
  delete b;
  return KDE_OK;
}

}  // extern "C"
