// Internal definitions shared by the library's translation units: status
// plumbing, workspace carving, launch geometry and small device helpers.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>

#include "../../include/kde.h"
#include "../../include/kde_measure.h"

namespace kde {

// ----------------------------------------------------------------- status

// Record a message for kde_last_error() on this thread and return `code`.
kde_status fail(kde_status code, const char* fmt, ...);
void clear_error();

#define KDE_TRY_HIP(expr)                                                          \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return ::kde::fail(KDE_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

#define KDE_CHECK_LAUNCH()                                                         \
  do {                                                                             \
    hipError_t _e = hipGetLastError();                                             \
    if (_e != hipSuccess)                                                          \
      return ::kde::fail(KDE_E_HIP, "kernel launch failed: %s", hipGetErrorString(_e)); \
  } while (0)

#define KDE_RETURN_IF(st)          \
  do {                             \
    kde_status _s = (st);          \
    if (_s != KDE_OK) return _s;   \
  } while (0)

// ------------------------------------------------------------- constants

constexpr int kBlock = 256;               // threads per workgroup for every kernel
constexpr int kCvTile = 256;              // particles per CV tile (one per thread)
constexpr int64_t kCvMaxSlots = 32768;    // rows of CV partial sums: tile pairs are dealt to this many slots
constexpr double kSkipExponent = 70.0;    // terms below exp(-70) of their sum's scale are skipped
constexpr int64_t kMaxN = int64_t(1) << 30;
constexpr int kMaxM = 4096;
constexpr int kProbeMaxBlocks = 65536;                // kde_probe_peak limits
constexpr int64_t kProbeMaxIters = int64_t(1) << 30;

// ------------------------------------------------------------ workspace

// Bump allocator over a caller-provided device buffer; every block is
// 256-byte aligned. In "measure" mode (base == nullptr) it only counts.
struct Carver {
  char* base;
  size_t cap;
  size_t used = 0;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool fits() const { return used <= cap; }
};

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------ timing

// Times one region of kernel launches when kernel timing is enabled
// (kde_timing_enable): the region's first launch records start() and its
// last launch stop() itself (hipExtLaunchKernelGGL), so the interval runs
// from the first kernel's start to the last kernel's end on the device and
// holds no host time before the first launch. When timing is off (or the
// stream is being captured) both are null and the launches record nothing.
class TimedLaunch {
 public:
  TimedLaunch(int id, hipStream_t s);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;
  hipEvent_t start() const { return start_; }
  // handing out the stop event marks the region as launched
  hipEvent_t stop() {
    armed_ = active_;
    return stop_;
  }

 private:
  int id_;
  hipStream_t s_;
  hipEvent_t start_{}, stop_{};
  bool active_ = false, armed_ = false;
};

// ----------------------------------------------------- argument checking

kde_status check_domain(const kde_domain* dom, bool need_grid);
// Fails (without launching) when a kernel would need more LDS per workgroup
// than the current device provides.
kde_status check_lds(size_t bytes);
kde_status check_workspace(void* ws, size_t ws_bytes, size_t need);
// The argument rules of kde_cv_scan, without its workspace.
kde_status check_cv_args(const kde_domain* dom, int64_t N, const void* x, int B, const double* kappas_h,
                         const double* cv);
size_t elem_size(int prec);

// Launch shape of the pair kernel for (precision, N): `chunk`
// concentrations per pass, `group` concentrations per work unit (a
// multiple of chunk; 0 = all of them).
struct PairTuning {
  int chunk;
  int group;
};
PairTuning tuned_pass(int prec, int64_t n);
kde_status set_tuning(int prec, int count, const int64_t* n_max, const int32_t* chunk, const int32_t* group);

// Calls f(std::integral_constant<int, BC>{}) with the pair kernel's pass
// size for `chunk`: 4, 8, or 16 in double. The float kernel holds a
// compensated pair of sums per concentration, which at 16 per pass does
// not fit its registers, so float has no pass of 16 (set_tuning refuses
// it).
template <typename T, typename F>
inline void with_pass_size(int chunk, F&& f) {
  if (chunk == 4) {
    f(std::integral_constant<int, 4>{});
  } else if constexpr (std::is_same<T, double>::value) {
    if (chunk == 16)
      f(std::integral_constant<int, 16>{});
    else
      f(std::integral_constant<int, 8>{});
  } else {
    f(std::integral_constant<int, 8>{});
  }
}

// Tile pairs of a CV scan over n particles, and the slots (rows of partial
// sums, one workgroup per slot and concentration group) they are dealt to.
inline int64_t cv_tile_pairs(int64_t n) {
  const int64_t t = (n + kCvTile - 1) / kCvTile;
  return t * (t + 1) / 2;
}
inline int64_t cv_slots(int64_t n) {
  const int64_t p = cv_tile_pairs(n);
  return p < kCvMaxSlots ? p : kCvMaxSlots;
}

// Concentrations per work unit, and units per tile pair, for B values.
inline int pair_group_size(const PairTuning& t, int B) { return (t.group > 0 && t.group < B) ? t.group : B; }
inline int pair_groups(const PairTuning& t, int B) {
  const int g = pair_group_size(t, B);
  return (B + g - 1) / g;
}

// ----------------------------------------------------- shared launch plans

// Counting sort of CV particles by angular cell.
struct SortPlan {
  int64_t n;
  int cells;       // angular cells
  int blocks;      // histogram/scatter blocks
  int64_t chunk;   // particles per block
};
SortPlan make_sort_plan(int64_t n);

// ------------------------------------------------------------- launchers

// Packed particle element of the pair kernels: for double, three values per
// particle (cos(pi w/L), sin(pi w/L), w) with w the wrapped position; for
// float, one 32-bit fixed-point phase round(w/L * 2^32) mod 2^32.
template <typename T>
struct Packed;
template <>
struct Packed<double> {
  using type = double;
  static constexpr int per_particle = 3;
};
template <>
struct Packed<float> {
  using type = uint32_t;
  static constexpr int per_particle = 1;
};

// Packed particle of the triangle-shape pair kernel: the wrapped position
// as a fraction of the period in double (the float form uses the 32-bit
// phase of Packed<float>).
struct FracPos {
  double f;
};
template <typename T>
struct TriPacked;
template <>
struct TriPacked<double> {
  using type = FracPos;
};
template <>
struct TriPacked<float> {
  using type = uint32_t;
};

// Wrap, pack and sort by cell, stably. `packed` receives n elements of P
// (one P per particle; the double half-angle form takes two doubles).
// Non-finite positions are noted in `status` (may be null).
template <typename T, typename P>
kde_status launch_pack_sorted_as(const T* x, int64_t n, double L, const SortPlan& plan, int32_t* hist, P* packed,
                                 int32_t* perm, hipStream_t s, uint32_t* status);
template <typename T>
inline kde_status launch_pack_sorted(const T* x, int64_t n, double L, const SortPlan& plan, int32_t* hist,
                                     typename Packed<T>::type* packed, int32_t* perm, hipStream_t s,
                                     uint32_t* status) {
  return launch_pack_sorted_as<T, typename Packed<T>::type>(x, n, L, plan, hist, packed, perm, s, status);
}

// One-set launchers of the path (cv.hip, density.hip); `status` receives
// KDE_NUMERIC_* bits (may be null).
size_t cv_workspace_bytes(int64_t n, int B, int prec);
kde_status cv_scan(const kde_domain* dom, int64_t n, const void* x, int B, const double* kappas, double* cv,
                   double* sums, int32_t* argmin, void* ws, size_t ws_bytes, hipStream_t s, uint32_t* status);
size_t deposit_workspace_bytes(int64_t n, int M);
size_t adapt_workspace_bytes(int64_t n);
kde_status deposit(const kde_domain* dom, int64_t n, const void* x, const void* kap, double kappa, double* rho,
                   void* ws, size_t ws_bytes, hipStream_t s, uint32_t* status);
kde_status gather(const kde_domain* dom, int64_t n, const void* x, const void* kap, double kappa,
                  const double* field, void* out, hipStream_t s, uint32_t* status);
kde_status adapt_widths(const kde_domain* dom, int64_t n, const void* x, const double* pilot, double kappa_star,
                        double alpha, void* kout, double* log_g, int64_t* nfl, void* ws, size_t ws_bytes,
                        hipStream_t s, uint32_t* status);

// Workspace of the Fourier-moment ops (KDE_OP_CV_FOURIER, _CV_REFINE,
// _ADAPT_EXACT), sized for the largest series order the ops accept.
size_t fourier_workspace_bytes(int op, int64_t n, int B);

// Deterministic column sums: out[c] = scale * sum_r in[r][c], fixed order.
// `scratch` must hold column_sum_scratch(rows, cols) bytes.
kde_status launch_column_sum(const double* in, int64_t rows, int cols, double* scratch,
                             double* out, hipStream_t s, double scale = 1.0);
size_t column_sum_scratch(int64_t rows, int cols);

// ----------------------------------------------------------- device helpers

// Numeric status words (KDE_NUMERIC_* bits). Kernels that read positions
// or per-particle concentrations note non-finite values (and concentrations
// outside their range) here: one atomic per wave and kind, taken by the
// wave's first lane that saw one; nothing else changes (outputs carry NaN).
// A null word records nothing. Lanes that are inactive at the call add
// nothing to the ballots.
__device__ __forceinline__ void note_numeric(uint32_t* status, bool bad_position, bool bad_concentration) {
  if (status == nullptr) return;
  const uint64_t mp = __ballot(bad_position);
  const uint64_t mc = __ballot(bad_concentration);
  const uint64_t any = mp | mc;
  if (any == 0) return;
  if (int(threadIdx.x & 63) == __ffsll((unsigned long long)any) - 1)
    atomicOr(status, (mp ? uint32_t(KDE_NUMERIC_POSITION) : 0u) | (mc ? uint32_t(KDE_NUMERIC_CONCENTRATION) : 0u));
}

// The plain calls' numeric status word on the current device (numeric.hip),
// or nullptr when it cannot be looked up (then nothing is recorded).
uint32_t* plain_numeric_word();

template <typename T>
__device__ __forceinline__ T wrap_position(T x, T L) {
  T y = x - L * floor(x / L);
  return (y >= L) ? T(0) : y;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

// Sum over the 64 lanes of a wave (butterfly; every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_d(v, m);
  return v;
}

}  // namespace kde
