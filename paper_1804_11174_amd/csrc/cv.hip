// Least-squares cross-validation over a batch of concentrations
// (Sec. II.B, Eq. cv_def): the O(N^2) pair sums and the final combination.
//
// For the von Mises kernel both pair terms depend on a pair only through
// its half-angle difference phi = pi (x_i - x_j) / L, via s = sin(phi) and
// c = |cos(phi)|:
//   K-term    exp(-2 kappa s^2)                           (kernel, unnormalised)
//   Kbar-term exp(-2 kappa (1 - c)) I0e(2 kappa c)        (two-fold convolution)
// Both exponents are formed without cancellation:
//   double: from half-angle vectors (a, b) = (cos(pi x/L), sin(pi x/L)),
//           c = |a_i a_j + b_i b_j|, s = b_i a_j - a_i b_j, 1 - c = s^2 / (1 + c);
//   float : from 32-bit fixed-point phases, whose wrapped integer difference
//           gives phi in [-pi/2, pi/2) exactly up to one conversion; then
//           1 - c = phi^2 R(phi^2) with R the Taylor series of
//           (1 - cos phi) / phi^2 (7 terms, below float rounding on that
//           range) and s^2 = (1 - c)(1 + c) = q (2 - q). Normalisers 1/(L I0e(kappa)) and
// 1/(L I0e(kappa)^2) are applied once, in double, by the finalize kernel.
//
// Work decomposition: particles (sorted by angular cell) are cut into tiles
// of 256. A tile pair (I <= J) is taken one i-particle per thread against
// the J tile staged in LDS (every lane reads the same j: an LDS
// broadcast). Concentrations are processed in chunks of up to 16, each with
// per-thread accumulators; at the end of a chunk the 256 per-thread sums
// are reduced in double in a fixed order into the workgroup's running
// sums. A workgroup owns one slot: the tile pairs k = slot, slot + S, ...
// of the list ordered by circular tile distance (pair_decode), S =
// min(tile pairs, 32768), and writes the slot's 2B sums to its own row, so
// the partial sums take at most 32768 x 2B doubles at any N. No
// floating-point atomics are used.
//
// Terms whose exponent is below -70 are not evaluated: each is below
// e^-70 (4e-31) times the largest term of its sum (the pair at distance 0
// has exponent 0 and I0e <= 1). Concentrations are ascending and the
// exponent scales with kappa, so once every lane of a wave is below the
// bound for one concentration, the wave skips the rest for that j.
//
// The first-order (triangular) shape of adjustable width (dev_tri.hpp)
// takes the same path: sort, tile pairs, fixed-order sums, finalize, with
// its own pair function and normalisation; the candidates are half-widths.
#include <climits>
#include <mutex>
#include <vector>

#include "dev_cv.hpp"
#include "dev_tri.hpp"

namespace kde {

// Triangle shape: one workgroup per slot (cv_slots(n) of them), compiled
// for eight waves per SIMD, which the tile-pair body fits on its own (the
// loop over a slot's tile pairs otherwise keeps more values live).
template <typename T, int BC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) tri_pairs_kernel(const typename TriPacked<T>::type* __restrict__ packed,
                                                          int64_t n, int cells, int64_t nslots, TriConsts<T> K,
                                                          double* __restrict__ partials) {
  __shared__ TriSmem<T, BC> sm;
  tri_slot<T, BC>(packed, n, cells, int64_t(blockIdx.x), nslots, K, partials + int64_t(blockIdx.x) * 2 * K.B, sm);
}

// raw[0..B): 3 h Tbar / 4 sums, raw[B..2B): h T sums; widths h_b. One
// block. S1 = raw1 / (3 h / 4), S2 = raw2 / h, Tbar(0) = 2 / (3 h); the objective and
// its first minimum as for the von Mises kernel.
__global__ void __launch_bounds__(KDE_MAX_KAPPAS) tri_finalize_kernel(const double* __restrict__ raw, int B,
                                                                     double n, KappaList widths,
                                                                     double* __restrict__ cv,
                                                                     double* __restrict__ sums,
                                                                     int32_t* __restrict__ argmin) {
  __shared__ double v[KDE_MAX_KAPPAS];
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const double h = widths.k[b];
    const double S1 = raw[b] / (0.75 * h);
    const double S2 = raw[B + b] / h;
    const double val = (n * (2.0 / (3.0 * h)) + 2.0 * S1) / (n * n) - 4.0 * S2 / (n * (n - 1.0));
    if (cv) cv[b] = val;
    v[b] = val;
    if (sums) {
      sums[b] = S1;
      sums[B + b] = S2;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && argmin) {
    int best = 0;
    for (int t = 1; t < B; ++t)
      if (v[t] < v[best]) best = t;
    *argmin = best;
  }
}

// Block (slot r, concentration group g) with r = blockIdx.x / groups.
template <typename T, int BC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(PairWaves<T, BC>::value))) cv_pairs_kernel(const typename Packed<T>::type* __restrict__ packed,
                                                         int64_t n, int cells, double L, int64_t nslots, int groups,
                                                         int gsize, CvConsts<T> K, double* __restrict__ partials) {
  __shared__ CvSmem<T, BC> sm;
  const int64_t r = int64_t(blockIdx.x) / groups;
  const int g = int(int64_t(blockIdx.x) - r * groups);
  const int b_lo = g * gsize;
  cv_slot<T, BC>(packed, n, cells, L, r, nslots, K, b_lo, min(K.B, b_lo + gsize), partials + r * 2 * K.B, sm);
}

// raw[0..B): Kbar sums, raw[B..2B): K sums (unnormalised); one block.
__global__ void __launch_bounds__(KDE_MAX_KAPPAS) cv_finalize_kernel(const double* __restrict__ raw, int B,
                                                                    double n, double L, KappaList kap,
                                                                    double* __restrict__ cv,
                                                                    double* __restrict__ sums,
                                                                    int32_t* __restrict__ argmin) {
  __shared__ double v[KDE_MAX_KAPPAS];
  cv_finalize_block(raw, B, n, L, kap, cv, sums, argmin, v, nullptr);
}

// ------------------------------------------------------------------ host

// Launch shape of the pair kernel, by precision and particle count
// (kde_tune_set): concentrations per pass and per work unit. The
// per-concentration sums do not depend on either: each concentration
// accumulates the same terms in the same order and the skip test is
// monotone in kappa. The defaults are the table the autotuner
// (paper_1804_11174_amd/autotune.py) measured on gfx950, written by it to
// tune_gfx950.inc.
namespace {
struct TuneEntry {
  int64_t n_max;
  PairTuning t;
};
std::mutex g_tune_mu;
#include "tune_gfx950.inc"
std::vector<TuneEntry> g_tune[2] = {KDE_TUNE_F64, KDE_TUNE_F32};
}  // namespace

PairTuning tuned_pass(int prec, int64_t n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneEntry& e : g_tune[prec]) if (n <= e.n_max) return e.t;
  return g_tune[prec].back().t;
}

kde_status set_tuning(int prec, int count, const int64_t* n_max, const int32_t* chunk, const int32_t* group) {
  std::vector<TuneEntry> t;
  for (int k = 0; k < count; ++k) {
    if (chunk[k] != 4 && chunk[k] != 8 && !(chunk[k] == 16 && prec == KDE_F64))
      return fail(KDE_E_INVALID_ARG, "chunk must be 4 or 8, or 16 in double (entry %d is %d)", k, chunk[k]);
    const int g = group ? group[k] : 0;
    if (g < 0 || g > KDE_MAX_KAPPAS || g % chunk[k] != 0)
      return fail(KDE_E_INVALID_ARG, "group must be 0 or a multiple of chunk up to %d (entry %d is %d)",
                  KDE_MAX_KAPPAS, k, g);
    if (k > 0 && !(n_max[k] > n_max[k - 1])) return fail(KDE_E_INVALID_ARG, "n_max must be strictly ascending");
    t.push_back(TuneEntry{n_max[k], PairTuning{chunk[k], g}});
  }
  t.back().n_max = INT64_MAX;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[prec] = t;
  return KDE_OK;
}

struct CvPlan {
  SortPlan sort;
  int64_t slots;  // rows of partial sums
};

static CvPlan make_cv_plan(int64_t n) {
  CvPlan p;
  p.sort = make_sort_plan(n);
  p.slots = cv_slots(n);
  return p;
}

struct CvBuffers {
  int32_t* hist;
  void* packed;
  double* partials;
  double* colsum;
  double* raw;
};

static CvBuffers carve_cv(Carver& cv, const CvPlan& p, int64_t n, int B, int prec) {
  CvBuffers b;
  b.hist = cv.take<int32_t>(size_t(p.sort.cells) * p.sort.blocks);
  b.packed = prec == KDE_F64 ? static_cast<void*>(cv.take<double>(Packed<double>::per_particle * size_t(n)))
                             : static_cast<void*>(cv.take<uint32_t>(size_t(n)));
  b.partials = cv.take<double>(size_t(p.slots) * 2 * B);
  b.colsum = cv.take<double>(column_sum_scratch(p.slots, 2 * B) / sizeof(double) + 1);
  b.raw = cv.take<double>(2 * size_t(B));
  return b;
}

size_t cv_workspace_bytes(int64_t n, int B, int prec) {
  CvPlan p = make_cv_plan(n);
  Carver c(nullptr, 0);
  carve_cv(c, p, n, B, prec);
  return c.used;
}

template <typename T>
static kde_status run_cv(const kde_domain* dom, int64_t n, const T* x, int B, const double* kappas,
                         double* cv, double* sums, int32_t* argmin, void* ws, size_t ws_bytes,
                         hipStream_t s, uint32_t* status) {
  CvPlan p = make_cv_plan(n);
  Carver c(ws, ws_bytes);
  CvBuffers buf = carve_cv(c, p, n, B, dom->prec);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.used);
  using P = typename Packed<T>::type;
  P* packed = static_cast<P*>(buf.packed);
  KDE_RETURN_IF(launch_pack_sorted<T>(x, n, dom->L, p.sort, buf.hist, packed, nullptr, s, status));
  CvConsts<T> K = make_consts<T>(kappas, B);
  const PairTuning tp = tuned_pass(dom->prec, n);
  const int groups = pair_groups(tp, B), gsize = pair_group_size(tp, B);
  {
    TimedLaunch timed(KDE_KERNEL_CV_PAIRS, s);
    const dim3 grid{unsigned(p.slots * groups)}, block{unsigned(kBlock)};
    with_pass_size<T>(tp.chunk, [&](auto bc) {
      hipExtLaunchKernelGGL((cv_pairs_kernel<T, decltype(bc)::value>), grid, block, 0, s, timed.start(),
                            timed.stop(), 0, (const P*)packed, n, p.sort.cells, dom->L, p.slots, groups, gsize, K,
                            buf.partials);
    });
  }
  KDE_CHECK_LAUNCH();
  KDE_RETURN_IF(launch_column_sum(buf.partials, p.slots, 2 * B, buf.colsum, buf.raw, s));
  const KappaList kl = make_kappa_list<T>(kappas, B);
  hipLaunchKernelGGL(cv_finalize_kernel, dim3(1), dim3(KDE_MAX_KAPPAS), 0, s, (const double*)buf.raw, B,
                     double(n), dom->L, kl, cv, sums, argmin);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

// Passes of the triangle pair kernel: widths per pass, 4 in both
// precisions. In float the three registers of each compensated sum make a
// pass of 8 spill at eight waves, and at five or six it runs slower (5.0
// against 4.4 ms at the paper-scale scan); in double 4 runs 4 % faster
// than 8 (6.93 against 7.19 ms).
template <typename T>
constexpr int kTriPass = 4;

template <typename T>
static kde_status run_cv_tri(const kde_domain* dom, int64_t n, const T* x, int B, const double* widths,
                             double* cv, double* sums, int32_t* argmin, void* ws, size_t ws_bytes, hipStream_t s,
                             uint32_t* status) {
  CvPlan p = make_cv_plan(n);
  Carver c(ws, ws_bytes);
  CvBuffers buf = carve_cv(c, p, n, B, dom->prec);
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, c.used);
  using P = typename TriPacked<T>::type;
  P* packed = static_cast<P*>(buf.packed);
  KDE_RETURN_IF((launch_pack_sorted_as<T, P>(x, n, dom->L, p.sort, buf.hist, packed, nullptr, s, status)));
  const TriConsts<T> K = make_tri_consts<T>(widths, B, dom->L);
  {
    TimedLaunch timed(KDE_KERNEL_CV_PAIRS, s);
    hipExtLaunchKernelGGL((tri_pairs_kernel<T, kTriPass<T>>), dim3(unsigned(p.slots)), dim3(kBlock), 0, s,
                          timed.start(), timed.stop(), 0, (const P*)packed, n, p.sort.cells, p.slots, K,
                          buf.partials);
  }
  KDE_CHECK_LAUNCH();
  KDE_RETURN_IF(launch_column_sum(buf.partials, p.slots, 2 * B, buf.colsum, buf.raw, s));
  KappaList kl{};
  for (int b = 0; b < B; ++b) kl.k[b] = widths[b];
  hipLaunchKernelGGL(tri_finalize_kernel, dim3(1), dim3(KDE_MAX_KAPPAS), 0, s, (const double*)buf.raw, B, double(n),
                     kl, cv, sums, argmin);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

kde_status cv_scan(const kde_domain* dom, int64_t n, const void* x, int B, const double* kappas, double* cv,
                   double* sums, int32_t* argmin, void* ws, size_t ws_bytes, hipStream_t s, uint32_t* status) {
  if (dom->shape == KDE_SHAPE_TRIANGLE) {
    if (dom->prec == KDE_F64)
      return run_cv_tri<double>(dom, n, static_cast<const double*>(x), B, kappas, cv, sums, argmin, ws, ws_bytes, s,
                                status);
    return run_cv_tri<float>(dom, n, static_cast<const float*>(x), B, kappas, cv, sums, argmin, ws, ws_bytes, s,
                             status);
  }
  if (dom->prec == KDE_F64)
    return run_cv<double>(dom, n, static_cast<const double*>(x), B, kappas, cv, sums, argmin, ws, ws_bytes, s,
                          status);
  return run_cv<float>(dom, n, static_cast<const float*>(x), B, kappas, cv, sums, argmin, ws, ws_bytes, s, status);
}

}  // namespace kde
