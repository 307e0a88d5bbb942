// The library's C ABI (include/kde.h): argument validation on the host,
// workspace sizing, and dispatch to the kernels. Nothing is enqueued when a
// check fails; the message is kept per thread for kde_last_error().
#include <cmath>
#include <cstring>

#include "kde_internal.hpp"

namespace kde {

static thread_local char g_err[512];

kde_status fail(kde_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = 0; }

size_t elem_size(int prec) { return prec == KDE_F64 ? sizeof(double) : sizeof(float); }

kde_status check_domain(const kde_domain* dom, bool need_grid) {
  if (!dom) return fail(KDE_E_INVALID_ARG, "domain pointer is NULL");
  if (!std::isfinite(dom->L) || !(dom->L > 0.0)) return fail(KDE_E_INVALID_ARG, "L must be finite and > 0 (got %g)", dom->L);
  if (dom->prec != KDE_F64 && dom->prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32 (got %d)", dom->prec);
  if (need_grid && (dom->M < 2 || dom->M > kMaxM)) return fail(KDE_E_INVALID_ARG, "M must lie in [2, %d] (got %d)", kMaxM, dom->M);
  if (dom->shape != KDE_SHAPE_VONMISES && dom->shape != KDE_SHAPE_TRIANGLE)
    return fail(KDE_E_INVALID_ARG, "shape must be KDE_SHAPE_VONMISES or KDE_SHAPE_TRIANGLE (got %d)", dom->shape);
  return KDE_OK;
}

kde_status check_workspace(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return KDE_OK;
  if (!ws) return fail(KDE_E_WORKSPACE, "workspace pointer is NULL (%zu bytes needed)", need);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(KDE_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(KDE_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return KDE_OK;
}

kde_status check_lds(size_t bytes) {
  static thread_local int cached_dev = -1;
  static thread_local int cached_lds = 0;
  int dev = 0;
  KDE_TRY_HIP(hipGetDevice(&dev));
  if (dev != cached_dev) {
    int v = 0;
    KDE_TRY_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    cached_dev = dev;
    cached_lds = v;
  }
  if (bytes > size_t(cached_lds))
    return fail(KDE_E_INVALID_ARG, "grid of this size needs %zu bytes of LDS per workgroup; the device offers %d",
                bytes, cached_lds);
  return KDE_OK;
}

static kde_status check_n(int64_t N, int64_t lo) {
  if (N < lo || N > kMaxN) return fail(KDE_E_INVALID_ARG, "N must lie in [%lld, %lld] (got %lld)", (long long)lo, (long long)kMaxN, (long long)N);
  return KDE_OK;
}

// A shape parameter: a concentration >= 0, or a triangle half-width in (0, L/2].
static kde_status check_kappa(const kde_domain* dom, double k, const char* what) {
  if (dom->shape == KDE_SHAPE_TRIANGLE) {
    if (!std::isfinite(k) || !(k > 0.0) || k > 0.5 * dom->L)
      return fail(KDE_E_INVALID_ARG, "%s (a half-width) must lie in (0, L/2] (got %g)", what, k);
    return KDE_OK;
  }
  if (!std::isfinite(k) || k < 0.0) return fail(KDE_E_INVALID_ARG, "%s must be finite and >= 0 (got %g)", what, k);
  return KDE_OK;
}

kde_status check_cv_args(const kde_domain* dom, int64_t N, const void* x, int B, const double* kappas_h,
                         const double* cv) {
  KDE_RETURN_IF(check_domain(dom, false));
  KDE_RETURN_IF(check_n(N, 2));
  if (B < 1 || B > KDE_MAX_KAPPAS) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d] (got %d)", KDE_MAX_KAPPAS, B);
  if (!x || !cv) return fail(KDE_E_INVALID_ARG, "x and cv must not be NULL");
  if (!kappas_h) return fail(KDE_E_INVALID_ARG, "kappas_h is NULL");
  for (int b = 0; b < B; ++b) {
    KDE_RETURN_IF(check_kappa(dom, kappas_h[b], "every kappa"));
    if (dom->shape == KDE_SHAPE_VONMISES && kappas_h[b] > KDE_MAX_CV_KAPPA)
      return fail(KDE_E_INVALID_ARG, "every kappa must be <= %g (got %g)", KDE_MAX_CV_KAPPA, kappas_h[b]);
    if (b > 0 && !(kappas_h[b] > kappas_h[b - 1])) return fail(KDE_E_INVALID_ARG, "kappas must be strictly ascending (index %d)", b);
  }
  return KDE_OK;
}

}  // namespace kde

using namespace kde;

extern "C" {

int32_t kde_abi_version(void) { return KDE_ABI_VERSION; }

const char* kde_status_str(kde_status s) {
  switch (s) {
    case KDE_OK: return "ok";
    case KDE_E_INVALID_ARG: return "invalid argument";
    case KDE_E_WORKSPACE: return "workspace missing or too small";
    case KDE_E_BUDGET: return "request exceeds budget";
    case KDE_E_AGAIN: return "not ready";
    case KDE_E_NOT_FOUND: return "unknown handle or ticket";
    case KDE_E_HIP: return "HIP runtime error";
    case KDE_E_NUMERIC: return "non-finite value";
    case KDE_E_INTERNAL: return "internal error";
    case KDE_E_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

const char* kde_last_error(void) { return g_err; }

kde_status kde_workspace_size(int32_t op, const kde_domain* dom, int64_t N, int32_t B, size_t* bytes_h) {
  clear_error();
  if (!bytes_h) return fail(KDE_E_INVALID_ARG, "bytes_h is NULL");
  switch (op) {
    case KDE_OP_CV_SCAN:
      KDE_RETURN_IF(check_domain(dom, false));
      KDE_RETURN_IF(check_n(N, 2));
      if (B < 1 || B > KDE_MAX_KAPPAS) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d] (got %d)", KDE_MAX_KAPPAS, B);
      *bytes_h = cv_workspace_bytes(N, B, dom->prec);
      return KDE_OK;
    case KDE_OP_DEPOSIT:
      KDE_RETURN_IF(check_domain(dom, true));
      KDE_RETURN_IF(check_n(N, 1));
      *bytes_h = deposit_workspace_bytes(N, dom->M);
      return KDE_OK;
    case KDE_OP_GATHER:
      KDE_RETURN_IF(check_domain(dom, true));
      KDE_RETURN_IF(check_n(N, 1));
      *bytes_h = 0;
      return KDE_OK;
    case KDE_OP_ADAPT:
      KDE_RETURN_IF(check_domain(dom, true));
      KDE_RETURN_IF(check_n(N, 1));
      *bytes_h = adapt_workspace_bytes(N);
      return KDE_OK;
    case KDE_OP_CV_FOURIER:
    case KDE_OP_CV_REFINE:
      KDE_RETURN_IF(check_domain(dom, false));
      KDE_RETURN_IF(check_n(N, 2));
      if (B < 1 || B > KDE_MAX_KAPPAS) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d] (got %d)", KDE_MAX_KAPPAS, B);
      *bytes_h = fourier_workspace_bytes(op, N, B);
      return KDE_OK;
    case KDE_OP_ADAPT_EXACT:
      KDE_RETURN_IF(check_domain(dom, false));
      KDE_RETURN_IF(check_n(N, 1));
      *bytes_h = fourier_workspace_bytes(op, N, 0);
      return KDE_OK;
    default:
      return fail(KDE_E_INVALID_ARG, "unknown op %d", op);
  }
}

kde_status kde_tune_set(int32_t prec, int32_t count, const int64_t* n_max_h, const int32_t* chunk_h,
                        const int32_t* group_h) {
  clear_error();
  if (prec != KDE_F64 && prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32");
  if (count < 1 || count > 64 || !n_max_h || !chunk_h)
    return fail(KDE_E_INVALID_ARG, "count must lie in [1, 64] with n_max and chunk given");
  return set_tuning(prec, count, n_max_h, chunk_h, group_h);
}

kde_status kde_tune_get(int32_t prec, int64_t N, int32_t* chunk_h, int32_t* group_h) {
  clear_error();
  if (prec != KDE_F64 && prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32");
  if (!chunk_h) return fail(KDE_E_INVALID_ARG, "chunk_h is NULL");
  const PairTuning t = tuned_pass(prec, N);
  *chunk_h = t.chunk;
  if (group_h) *group_h = t.group;
  return KDE_OK;
}

kde_status kde_cv_scan(const kde_domain* dom, int64_t N, const void* x, int32_t B, const double* kappas_h,
                       double* cv, double* sums, int32_t* argmin, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  KDE_RETURN_IF(check_cv_args(dom, N, x, B, kappas_h, cv));
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, cv_workspace_bytes(N, B, dom->prec)));
  return cv_scan(dom, N, x, B, kappas_h, cv, sums, argmin, ws, ws_bytes, static_cast<hipStream_t>(stream),
                 plain_numeric_word());
}

kde_status kde_deposit(const kde_domain* dom, int64_t N, const void* x, const void* kappa_i, double kappa,
                       double* rho, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  KDE_RETURN_IF(check_domain(dom, true));
  KDE_RETURN_IF(check_n(N, 1));
  if (!x || !rho) return fail(KDE_E_INVALID_ARG, "x and rho must not be NULL");
  if (!kappa_i) KDE_RETURN_IF(check_kappa(dom, kappa, "kappa"));
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, deposit_workspace_bytes(N, dom->M)));
  return deposit(dom, N, x, kappa_i, kappa, rho, ws, ws_bytes, static_cast<hipStream_t>(stream),
                 plain_numeric_word());
}

kde_status kde_gather(const kde_domain* dom, int64_t N, const void* x, const void* kappa_i, double kappa,
                      const double* field, void* out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  (void)ws;
  (void)ws_bytes;
  KDE_RETURN_IF(check_domain(dom, true));
  KDE_RETURN_IF(check_n(N, 1));
  if (!x || !field || !out) return fail(KDE_E_INVALID_ARG, "x, field and out must not be NULL");
  if (!kappa_i) KDE_RETURN_IF(check_kappa(dom, kappa, "kappa"));
  return gather(dom, N, x, kappa_i, kappa, field, out, static_cast<hipStream_t>(stream), plain_numeric_word());
}

kde_status kde_adapt_widths(const kde_domain* dom, int64_t N, const void* x, const double* pilot,
                            double kappa_star, double alpha, void* kappa_out, double* log_geomean,
                            int64_t* n_floored, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  KDE_RETURN_IF(check_domain(dom, true));
  KDE_RETURN_IF(check_n(N, 1));
  if (dom->shape != KDE_SHAPE_VONMISES) return fail(KDE_E_INVALID_ARG, "adaptive widths are defined for the von Mises shape");
  if (!x || !pilot || !kappa_out) return fail(KDE_E_INVALID_ARG, "x, pilot and kappa_out must not be NULL");
  if (!std::isfinite(kappa_star) || !(kappa_star > 0.0)) return fail(KDE_E_INVALID_ARG, "kappa_star must be finite and > 0 (got %g)", kappa_star);
  if (!std::isfinite(alpha) || alpha < 0.0) return fail(KDE_E_INVALID_ARG, "alpha must be finite and >= 0 (got %g)", alpha);
  KDE_RETURN_IF(check_workspace(ws, ws_bytes, adapt_workspace_bytes(N)));
  return adapt_widths(dom, N, x, pilot, kappa_star, alpha, kappa_out, log_geomean, n_floored, ws, ws_bytes,
                      static_cast<hipStream_t>(stream), plain_numeric_word());
}

}  // extern "C"
