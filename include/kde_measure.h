/*
 * kde_measure.h -- measurement hooks of libkdepic.so, for benchmarks and
 * profiles only (no step of the KDE path needs them): per-kernel HIP-event
 * timing and issue-rate probes. The library exports them beside the calls
 * of kde.h; conventions (status codes, streams, memory) are those of kde.h.
 */
#ifndef KDE_MEASURE_H
#define KDE_MEASURE_H

#include "kde.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Kernel timing (diagnostics). While enabled, the library brackets every
 * launch of the kernels named below with a pair of HIP events recorded on
 * the launching call's stream. kde_timing_read waits for the recorded
 * events, adds their elapsed times to the kernel's running total and
 * returns it with the number of launches; kde_timing_reset clears all
 * totals. Events are host-side HIP objects: no device memory is
 * allocated. Enabling costs two event records per bracketed launch.
 */
enum kde_kernel_id {
  KDE_KERNEL_CV_PAIRS = 0,   /* the O(N^2) pair-sum kernel of kde_cv_scan   */
  KDE_KERNEL_DEPOSIT = 1,    /* the per-chunk grid kernel of kde_deposit     */
  KDE_KERNEL_GATHER = 2,     /* the per-particle kernel of kde_gather        */
  KDE_KERNEL_ADAPT = 3,      /* both per-particle passes of kde_adapt_widths */
  KDE_KERNEL_MOMENTS = 4,    /* the Fourier-moment kernel of the Fourier ops  */
  KDE_KERNEL_PROBE = 5,      /* the kernel of kde_probe_peak                  */
  KDE_KERNEL_COUNT = 6
};
kde_status kde_timing_enable(int32_t on);
kde_status kde_timing_reset(void);
kde_status kde_timing_read(int32_t kernel_id, double* total_ms_h, int64_t* launches_h);

/*
 * kde_probe_peak -- issue-rate probe (diagnostics, for pricing rooflines on
 * the device at hand rather than from its datasheet). Launches `blocks`
 * workgroups of 256 threads; every thread runs 8 independent dependency
 * chains of `iters` steps of one instruction kind and writes the sum of its
 * chains to out[thread]. Timed with kde_timing_* under KDE_KERNEL_PROBE,
 * the sustained rate is blocks x 256 x 8 x iters lane-operations per
 * elapsed second (an FMA counts as one).
 *   kind   : KDE_PROBE_FMA_F64 (double FMA), KDE_PROBE_FMA_F32 (float FMA,
 *            not packed), KDE_PROBE_EXP_F32 (the hardware base-2
 *            exponential), KDE_PROBE_ADD_F64 (double add).
 *   blocks : 1 .. 65536.
 *   iters  : a multiple of 4 in [4, 2^30].
 *   out    : device, blocks x 256 doubles (written; values are meaningless).
 * Errors: KDE_E_INVALID_ARG for an unknown kind, NULL out or sizes out of
 * range (nothing is launched).
 */
enum kde_probe_kind {
  KDE_PROBE_FMA_F64 = 0,
  KDE_PROBE_FMA_F32 = 1,
  KDE_PROBE_EXP_F32 = 2,
  KDE_PROBE_ADD_F64 = 3
};
kde_status kde_probe_peak(int32_t kind, int32_t blocks, int64_t iters, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KDE_MEASURE_H */
