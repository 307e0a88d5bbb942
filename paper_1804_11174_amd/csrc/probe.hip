// Issue-rate probes (kde_probe_peak in include/kde_measure.h): one kernel per
// instruction kind in which every thread runs kChains independent
// dependency chains of `iters` steps, so the device's sustained
// lane-operation rate for that kind is (threads x kChains x iters) / time.
// The chains are contractions or bounded maps (x -> a x + b with |a| < 1,
// x -> 2^-x, x -> x + b with a tiny b), so every value stays finite, and
// each thread writes the sum of its chains so nothing is optimised away.
#include "kde_internal.hpp"

namespace kde {

namespace {

constexpr int kChains = 8;

template <int KIND>
__global__ void __launch_bounds__(kBlock) probe_kernel(int64_t iters, double* __restrict__ out) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const double seed = 1.0 + 1e-3 * double(t & 7);
  double res = 0.0;
  if constexpr (KIND == KDE_PROBE_FMA_F64 || KIND == KDE_PROBE_ADD_F64) {
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + 1e-4 * c;
    const double a = 0.9999999, b = 1e-7;
    for (int64_t i = 0; i < iters; i += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = (KIND == KDE_PROBE_FMA_F64) ? fma(x[c], a, b) : x[c] + b;
      }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res += x[c];
  } else {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = float(seed) + 1e-4f * c;
    const float a = 0.9999f, b = 1e-4f;
    for (int64_t i = 0; i < iters; i += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
          x[c] = (KIND == KDE_PROBE_FMA_F32) ? fmaf(x[c], a, b) : __builtin_amdgcn_exp2f(-x[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) res += double(x[c]);
  }
  out[t] = res;
}

}  // namespace

}  // namespace kde

using namespace kde;

extern "C" {

kde_status kde_probe_peak(int32_t kind, int32_t blocks, int64_t iters, double* out, void* stream) {
  clear_error();
  if (!out) return fail(KDE_E_INVALID_ARG, "out must not be NULL");
  if (blocks < 1 || blocks > kProbeMaxBlocks)
    return fail(KDE_E_INVALID_ARG, "blocks must lie in [1, %d] (got %d)", kProbeMaxBlocks, blocks);
  if (iters < 4 || iters > kProbeMaxIters || iters % 4 != 0)
    return fail(KDE_E_INVALID_ARG, "iters must be a multiple of 4 in [4, %lld] (got %lld)",
                (long long)kProbeMaxIters, (long long)iters);
  if (kind < KDE_PROBE_FMA_F64 || kind > KDE_PROBE_ADD_F64) return fail(KDE_E_INVALID_ARG, "unknown probe kind %d", kind);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid{unsigned(blocks)}, block{unsigned(kBlock)};
  TimedLaunch timed(KDE_KERNEL_PROBE, s);
  switch (kind) {
    case KDE_PROBE_FMA_F64: hipExtLaunchKernelGGL(probe_kernel<KDE_PROBE_FMA_F64>, grid, block, 0, s, timed.start(), timed.stop(), 0, iters, out); break;
    case KDE_PROBE_FMA_F32: hipExtLaunchKernelGGL(probe_kernel<KDE_PROBE_FMA_F32>, grid, block, 0, s, timed.start(), timed.stop(), 0, iters, out); break;
    case KDE_PROBE_EXP_F32: hipExtLaunchKernelGGL(probe_kernel<KDE_PROBE_EXP_F32>, grid, block, 0, s, timed.start(), timed.stop(), 0, iters, out); break;
    case KDE_PROBE_ADD_F64: hipExtLaunchKernelGGL(probe_kernel<KDE_PROBE_ADD_F64>, grid, block, 0, s, timed.start(), timed.stop(), 0, iters, out); break;
    default: break;
  }
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

}  // extern "C"
