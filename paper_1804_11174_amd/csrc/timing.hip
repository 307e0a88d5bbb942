// Optional per-kernel timing with HIP events (kde_timing_* in include/kde_measure.h),
// recorded by the timed launches themselves. Pending event pairs are kept
// per kernel id; reading waits for them and folds their durations into
// running totals.
#include <mutex>
#include <vector>

#include "kde_internal.hpp"

namespace kde {

namespace {
struct Pending {
  hipEvent_t start, stop;
};
struct Slot {
  std::vector<Pending> pending;
  double total_ms = 0.0;
  int64_t launches = 0;
};
std::mutex g_mu;
bool g_on = false;
Slot g_slots[KDE_KERNEL_COUNT];
}  // namespace

TimedLaunch::TimedLaunch(int id, hipStream_t s) : id_(id), s_(s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || id < 0 || id >= KDE_KERNEL_COUNT) return;
  // a launch being captured into a graph is not timed (its events would be
  // recorded into the graph, not now)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&start_) != hipSuccess) {
    start_ = nullptr;
    return;
  }
  if (hipEventCreate(&stop_) != hipSuccess) {
    (void)hipEventDestroy(start_);
    start_ = stop_ = nullptr;
    return;
  }
  active_ = true;
}

TimedLaunch::~TimedLaunch() {
  if (!active_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!armed_) {  // nothing was launched with the events
    (void)hipEventDestroy(start_);
    (void)hipEventDestroy(stop_);
    return;
  }
  g_slots[id_].pending.push_back(Pending{start_, stop_});
}

}  // namespace kde

using namespace kde;

extern "C" {

kde_status kde_timing_enable(int32_t on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return KDE_OK;
}

kde_status kde_timing_reset(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& s : g_slots) {
    for (auto& p : s.pending) {
      (void)hipEventSynchronize(p.stop);
      (void)hipEventDestroy(p.start);
      (void)hipEventDestroy(p.stop);
    }
    s.pending.clear();
    s.total_ms = 0.0;
    s.launches = 0;
  }
  return KDE_OK;
}

kde_status kde_timing_read(int32_t kernel_id, double* total_ms_h, int64_t* launches_h) {
  clear_error();
  if (kernel_id < 0 || kernel_id >= KDE_KERNEL_COUNT) return fail(KDE_E_INVALID_ARG, "unknown kernel id %d", kernel_id);
  if (!total_ms_h || !launches_h) return fail(KDE_E_INVALID_ARG, "output pointers must not be NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  Slot& s = g_slots[kernel_id];
  kde_status st = KDE_OK;
  for (auto& p : s.pending) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(p.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
    if (e != hipSuccess && st == KDE_OK) st = fail(KDE_E_HIP, "timing event: %s", hipGetErrorString(e));
    s.total_ms += double(ms);
    s.launches += 1;
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  s.pending.clear();
  *total_ms_h = s.total_ms;
  *launches_h = s.launches;
  return st;
}

}  // extern "C"
