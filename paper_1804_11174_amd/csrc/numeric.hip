// The numeric status word of the plain calls: one per device, a file-scope
// __device__ variable whose address is looked up once per device (that
// device current) and passed to the kernels, which set KDE_NUMERIC_* bits
// in it (note_numeric). kde_numeric_check takes it with an atomic exchange.
#include <mutex>

#include "kde_internal.hpp"

namespace kde {

static __device__ uint32_t numeric_word;
static __device__ uint32_t numeric_taken;

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t* g_word[kMaxDevices] = {};
uint32_t* g_taken[kMaxDevices] = {};
}  // namespace

static kde_status lookup(int dev) {
  if (g_word[dev]) return KDE_OK;
  void* w = nullptr;
  void* t = nullptr;
  KDE_TRY_HIP(hipGetSymbolAddress(&w, HIP_SYMBOL(numeric_word)));
  KDE_TRY_HIP(hipGetSymbolAddress(&t, HIP_SYMBOL(numeric_taken)));
  g_word[dev] = static_cast<uint32_t*>(w);
  g_taken[dev] = static_cast<uint32_t*>(t);
  return KDE_OK;
}

uint32_t* plain_numeric_word() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (lookup(dev) != KDE_OK) return nullptr;
  return g_word[dev];
}

__global__ void numeric_take_kernel(uint32_t* word, uint32_t* taken) { *taken = atomicExch(word, 0u); }

}  // namespace kde

using namespace kde;

extern "C" kde_status kde_numeric_check(void* stream, uint32_t* flags_h) {
  clear_error();
  if (!flags_h) return fail(KDE_E_INVALID_ARG, "flags_h is NULL");
  int dev = 0;
  KDE_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(KDE_E_INTERNAL, "device index %d beyond %d", dev, kMaxDevices);
  uint32_t *w = nullptr, *t = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    KDE_RETURN_IF(lookup(dev));
    w = g_word[dev];
    t = g_taken[dev];
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(numeric_take_kernel, dim3(1), dim3(1), 0, s, w, t);
  KDE_CHECK_LAUNCH();
  KDE_TRY_HIP(hipStreamSynchronize(s));
  uint32_t v = 0;
  KDE_TRY_HIP(hipMemcpy(&v, t, sizeof v, hipMemcpyDeviceToHost));
  *flags_h = v;
  if (v) return fail(KDE_E_NUMERIC, "non-finite %s%s%s seen", (v & KDE_NUMERIC_POSITION) ? "positions" : "",
                     (v & KDE_NUMERIC_POSITION) && (v & KDE_NUMERIC_CONCENTRATION) ? " and " : "",
                     (v & KDE_NUMERIC_CONCENTRATION) ? "concentrations" : "");
  return KDE_OK;
}
