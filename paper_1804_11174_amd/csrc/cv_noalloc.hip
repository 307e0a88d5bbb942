// kde_cv_scan_noalloc: the CV scan of kde_cv_scan with its workspace in an
// array the library holds in device memory, for callers that cannot
// allocate (code under graph capture, serving loops, harnesses that forbid
// allocation). The kernels are kde_cv_scan's and take the array as their
// workspace, so the results are the same bits.
//
// The array is a file-scope __device__ variable: every device that runs a
// call holds its own copy, from the library's load on that device until
// the process ends. Host code never uses the variable's name as an
// address: on a device's first call its address is looked up with
// hipGetSymbolAddress (that device current) and kept per device. Every call
// on one device shares that device's array, so calls that overlap on one
// device (other streams, other threads) race; calls on one stream follow
// each other and are safe. Every byte a call reads from the array is
// written earlier in the same call (histograms, packed positions, slot
// sums, column sums), so nothing needs clearing between calls.
#include <mutex>

#include "kde_internal.hpp"

namespace kde {

static __device__ __align__(256) unsigned char scratch[KDE_CV_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device
}  // namespace

// The current device's copy of the array (looked up once per device).
static kde_status scratch_on_current_device(void** out) {
  int dev = 0;
  KDE_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(KDE_E_INTERNAL, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    KDE_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(KDE_E_INTERNAL, "no device address for the scratch array");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return KDE_OK;
}

}  // namespace kde

using namespace kde;

extern "C" {

kde_status kde_cv_scan_noalloc(const kde_domain* dom, int64_t N, const void* x, int32_t B, const double* kappas_h,
                               double* cv, double* sums, int32_t* argmin, void* stream) {
  clear_error();
  KDE_RETURN_IF(check_cv_args(dom, N, x, B, kappas_h, cv));
  const size_t need = cv_workspace_bytes(N, B, dom->prec);
  if (need > size_t(KDE_CV_NOALLOC_MAX_BYTES))
    return fail(KDE_E_WORKSPACE, "scan of N = %lld, B = %d needs %zu bytes of workspace; the library's array holds %zu",
                (long long)N, B, need, size_t(KDE_CV_NOALLOC_MAX_BYTES));
  void* ws = nullptr;
  KDE_RETURN_IF(scratch_on_current_device(&ws));
  return cv_scan(dom, N, x, B, kappas_h, cv, sums, argmin, ws, size_t(KDE_CV_NOALLOC_MAX_BYTES),
                 static_cast<hipStream_t>(stream), plain_numeric_word());
}

}  // extern "C"
