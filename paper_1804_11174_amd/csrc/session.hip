// Resident PIC sessions: the particle set stays in HBM across steps and
// every step runs the KDE-PIC cycle of Sec. III.A with the width-update
// rule of Sec. II.D (standard sessions run the same cycle with linear
// weighting and no width update, steps 1-4 only; both record the field
// energy of step 2 into a history):
//
//   1. deposit with the per-particle concentrations kappa_i;
//   2. Poisson solve and centred field on the grid (pic.hip);
//   3. gather of the field with kappa_i; 4. leapfrog push;
//   5. Anderson-Darling statistic of the new positions, read by the host,
//      which turns it into a p-value and applies the update rule:
//        p > 2 thr:          p_th = 2 thr;
//        p < p_th / 2:       CV scan (first n_cv particles) -> h_target, p_th = p;
//        always:             h_opt <- rate h_target + (1 - rate) h_opt;
//      then kappa* = (L / (2 pi h_opt))^2, a pilot deposit at kappa* and the
//      adaptive widths give the next step's kappa_i.
//
// The p-value is the upper tail of the limiting law of A^2 for a fully
// specified distribution, from Anderson and Darling's (1954) series; its
// integrals are done by the trapezoid rule after scaling out the Gaussian
// factor (the integrand is even and analytic, so the rule converges
// geometrically).
//
// A step is a small state machine, so that one thread can drive many
// sessions (the request server) without waiting on any: begin (enqueue the
// fixed part, whose last node copies A^2 and the numeric status word to a
// pinned mailbox, and record an event), then advance once that event has
// completed (apply the rule on the host; when it fires, enqueue the CV scan
// and record the event again; otherwise, or after the scan, enqueue the
// widths of the next step). kde_session_step runs the same machine,
// waiting on the event itself.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "session_internal.hpp"

namespace kde {

// implemented in pic.hip
size_t ad_workspace_bytes(int64_t n, int prec);
kde_status launch_poisson_field(const double* rho, int M, double L, double* E, hipStream_t s);
kde_status launch_field_energy(const double* E, int M, double L, double* energy, int64_t history, int64_t* step,
                               hipStream_t s);
kde_status launch_set_step(int64_t* step, int64_t value, hipStream_t s);
template <typename T>
kde_status launch_push(T* x, T* v, const T* E_i, int64_t n, double dt, double L, hipStream_t s);
template <typename T>
kde_status launch_ad_statistic(const T* x, int64_t n, double L, double* a2, void* ws, size_t ws_bytes, hipStream_t s);
size_t poisson_max_m();

// --------------------------------------------------------- AD p-value

static double ad_series_term(int j, double z) {
  // binom(-1/2, j) (4j+1) exp(-(4j+1)^2 pi^2 / (8z)) * I_j, with
  // I_j = int_0^inf exp(z / (8 (w^2 + 1)) - a w^2) dw, a = (4j+1)^2 pi^2 / (8z)
  double binom = 1.0;
  for (int k = 0; k < j; ++k) binom *= (-0.5 - k) / double(k + 1);
  const double c = double(4 * j + 1);
  const double a = c * c * M_PI * M_PI / (8.0 * z);
  // w = t / sqrt(a): I_j = a^(-1/2) int_0^inf exp(z / (8 (t^2/a + 1)) - t^2) dt,
  // whose integral is at most exp(z/8) sqrt(pi)/2: a term whose factor in
  // front makes that below 1e-30 is left out
  const double pre = binom * c * std::exp(-a) / std::sqrt(a);
  if (std::fabs(pre) * std::exp(z / 8.0) < 1e-30) return 0.0;
  // the integrand is analytic in the strip |Im t| < sqrt(a) (its
  // singularities are at t = +-i sqrt(a)), so the trapezoid rule converges
  // geometrically once the step is a small fraction of sqrt(a); with
  // h = min(0.05, sqrt(a)/20) the p-value agrees with an adaptive
  // quadrature of the same series to 1e-15 wherever p > 1e-15, at about a
  // fortieth of the points of a fixed step of 0.004
  const double h = std::fmin(0.05, std::sqrt(a) / 20.0);
  double s = 0.5 * std::exp(z / 8.0);
  for (int k = 1;; ++k) {
    const double t = k * h;
    s += std::exp(z / (8.0 * (t * t / a + 1.0)) - t * t);
    if (t > 9.0) break;
  }
  return pre * s * h;
}

double ad_upper_tail(double a2) {
  if (!(a2 > 0.0)) return 1.0;
  if (a2 > 200.0) return 0.0;
  double total = 0.0;
  for (int j = 0; j < 60; ++j) {
    const double t = ad_series_term(j, a2);
    total += t;
    if (j > 3 && std::fabs(t) < 1e-18) break;
  }
  double cdf = std::sqrt(2.0 * M_PI) / a2 * total;
  cdf = cdf < 0.0 ? 0.0 : (cdf > 1.0 ? 1.0 : cdf);
  return 1.0 - cdf;
}

// ------------------------------------------------------------- session

struct SessionState {
  int64_t step = 0;
  double p_th = 0.02, h_opt = 0.0, h_target = 0.0, kappa_star = 0.0;
  double last_a2 = 0.0, last_p = 1.0;
  int64_t fired = 0;
};

static double kappa_of_width(double h, double L) {
  const double r = L / (2.0 * M_PI * h);
  return r * r;
}
static double width_of_kappa(double k, double L) { return (L / (2.0 * M_PI)) / std::sqrt(k); }

}  // namespace kde

using namespace kde;

// Device and pinned-host mailbox of a session: the last A^2, the CV
// scan's first minimum and the numeric status word of the session's
// kernels, copied to the host together.
struct SessionMail {
  double a2;
  int32_t argmin;
  uint32_t status;
};

enum class StepPhase { Idle, Fixed, Scan };

struct kde_session {
  kde_pic_params prm{};
  std::vector<double> kappas;
  kde_domain dom{};
  kde_domain tdom{};  // triangle of half-width dx (standard sessions)
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;  // completion of the part of a step the host waits on
  size_t arena_bytes = 0;
  // device buffers in the arena
  void *x = nullptr, *v = nullptr, *kap = nullptr, *Ei = nullptr;
  double *rho = nullptr, *E = nullptr, *pilot = nullptr, *cv = nullptr, *energy = nullptr;
  SessionMail* dmail = nullptr;
  int64_t* step_dev = nullptr;  // history slot of the next field energy
  void* ws = nullptr;
  size_t ws_bytes = 0;
  SessionMail* mail = nullptr;  // pinned host copy of dmail
  // the step's fixed launch sequence, captured at the first step
  hipGraphExec_t fixed = nullptr;
  SessionState st;
  uint32_t numeric = 0;  // numeric status seen so far (sticky until a restore)
  StepPhase phase = StepPhase::Idle;
  std::chrono::steady_clock::time_point t_begin;
  ~kde_session() {
    if (fixed) (void)hipGraphExecDestroy(fixed);
    if (mail) (void)hipHostFree(mail);
    if (ev) (void)hipEventDestroy(ev);
  }
};

namespace kde {

static bool standard(const kde_pic_params& p) { return p.method == KDE_PIC_STANDARD; }

static size_t session_ws_bytes(const kde_pic_params& p) {
  if (standard(p)) return deposit_workspace_bytes(p.N, p.M);
  size_t w = cv_workspace_bytes(p.n_cv, p.B, p.prec);
  w = std::max(w, deposit_workspace_bytes(p.N, p.M));
  w = std::max(w, adapt_workspace_bytes(p.N));
  w = std::max(w, ad_workspace_bytes(p.N, p.prec));
  return w;
}

static size_t carve_session(Carver& c, const kde_pic_params& p, kde_session* s) {
  const size_t es = elem_size(p.prec);
  void* x = c.take<char>(size_t(p.N) * es);
  void* v = c.take<char>(size_t(p.N) * es);
  void* kap = c.take<char>(size_t(p.N) * es);
  void* Ei = c.take<char>(size_t(p.N) * es);
  double* rho = c.take<double>(p.M);
  double* E = c.take<double>(p.M);
  double* pilot = c.take<double>(p.M);
  double* cv = c.take<double>(standard(p) ? 1 : p.B);
  SessionMail* dmail = c.take<SessionMail>(1);
  double* energy = c.take<double>(size_t(std::max(p.history, 1)));
  int64_t* stepd = c.take<int64_t>(1);
  const size_t wsb = session_ws_bytes(p);
  void* ws = c.take<char>(wsb);
  if (s) {
    s->x = x; s->v = v; s->kap = kap; s->Ei = Ei;
    s->rho = rho; s->E = E; s->pilot = pilot; s->cv = cv; s->dmail = dmail;
    s->energy = energy;
    s->step_dev = stepd;
    s->ws = ws; s->ws_bytes = wsb;
  }
  return c.used;
}

static kde_status check_params(const kde_pic_params* p) {
  if (!p) return fail(KDE_E_INVALID_ARG, "params are NULL");
  if (p->N < 2 || p->N > kMaxN) return fail(KDE_E_INVALID_ARG, "N must lie in [2, %lld]", (long long)kMaxN);
  if (!std::isfinite(p->L) || !(p->L > 0.0)) return fail(KDE_E_INVALID_ARG, "L must be finite and > 0");
  if (p->M < 2 || size_t(p->M) > poisson_max_m() || (p->M & (p->M - 1)))
    return fail(KDE_E_INVALID_ARG, "M must be a power of two in [2, %zu]", poisson_max_m());
  if (p->prec != KDE_F64 && p->prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32");
  if (!std::isfinite(p->dt) || !(p->dt > 0.0)) return fail(KDE_E_INVALID_ARG, "dt must be finite and > 0");
  if (p->method != KDE_PIC_KDE && p->method != KDE_PIC_STANDARD)
    return fail(KDE_E_INVALID_ARG, "method must be KDE_PIC_KDE or KDE_PIC_STANDARD (got %d)", p->method);
  if (p->history < 0) return fail(KDE_E_INVALID_ARG, "history must be >= 0");
  if (standard(*p)) return KDE_OK;
  if (p->B < 1 || p->B > KDE_MAX_KAPPAS || !p->kappas_h) return fail(KDE_E_INVALID_ARG, "B must lie in [1, %d]", KDE_MAX_KAPPAS);
  for (int b = 0; b < p->B; ++b) {
    if (!std::isfinite(p->kappas_h[b]) || !(p->kappas_h[b] > 0.0) || p->kappas_h[b] > KDE_MAX_CV_KAPPA)
      return fail(KDE_E_INVALID_ARG, "kappas must lie in (0, %g]", KDE_MAX_CV_KAPPA);
    if (b > 0 && !(p->kappas_h[b] > p->kappas_h[b - 1])) return fail(KDE_E_INVALID_ARG, "kappas must be strictly ascending");
  }
  if (p->n_cv < 2 || p->n_cv > p->N) return fail(KDE_E_INVALID_ARG, "n_cv must lie in [2, N]");
  if (!std::isfinite(p->alpha) || p->alpha < 0.0) return fail(KDE_E_INVALID_ARG, "alpha must be finite and >= 0");
  if (!(p->p_threshold > 0.0 && p->p_threshold < 0.5)) return fail(KDE_E_INVALID_ARG, "p_threshold must lie in (0, 0.5)");
  if (!(p->adjust_rate > 0.0 && p->adjust_rate <= 1.0)) return fail(KDE_E_INVALID_ARG, "adjust_rate must lie in (0, 1]");
  return KDE_OK;
}

__global__ void session_clear_status_kernel(SessionMail* m) {
  if (threadIdx.x == 0) m->status = 0u;
}

static kde_status clear_status(kde_session* s) {
  hipLaunchKernelGGL(session_clear_status_kernel, dim3(1), dim3(64), 0, s->s, s->dmail);
  KDE_CHECK_LAUNCH();
  return KDE_OK;
}

static uint32_t* status_word(kde_session* s) { return &s->dmail->status; }

// Enqueue the CV scan on the first n_cv particles and the copy of the
// mailbox (first minimum, status) to the host.
static kde_status enqueue_cv(kde_session* s) {
  kde_domain d = s->dom;
  KDE_RETURN_IF(cv_scan(&d, s->prm.n_cv, s->x, s->prm.B, s->kappas.data(), s->cv, nullptr, &s->dmail->argmin,
                        s->ws, s->ws_bytes, s->s, status_word(s)));
  KDE_TRY_HIP(hipMemcpyAsync(s->mail, s->dmail, sizeof(SessionMail), hipMemcpyDeviceToHost, s->s));
  return KDE_OK;
}

// The scan's choice, from the host mailbox (its copy has completed).
static kde_status scanned_kappa(kde_session* s, double* kstar) {
  const int32_t b = s->mail->argmin;
  if (b < 0 || b >= s->prm.B) return fail(KDE_E_INTERNAL, "argmin out of range");
  *kstar = s->kappas[b];
  return KDE_OK;
}

// Pilot deposit at kappa* and the adaptive widths for the next step.
static kde_status session_widths(kde_session* s, double kstar) {
  KDE_RETURN_IF(deposit(&s->dom, s->prm.N, s->x, nullptr, kstar, s->pilot, s->ws, s->ws_bytes, s->s, status_word(s)));
  KDE_RETURN_IF(adapt_widths(&s->dom, s->prm.N, s->x, s->pilot, kstar, s->prm.alpha, s->kap, nullptr, nullptr, s->ws,
                             s->ws_bytes, s->s, status_word(s)));
  return KDE_OK;
}

static kde_status record_energy(kde_session* s) {
  return launch_field_energy(s->E, s->prm.M, s->prm.L, s->energy, s->prm.history, s->step_dev, s->s);
}

static kde_status push_any(kde_session* s) {
  const kde_pic_params& p = s->prm;
  if (p.prec == KDE_F64)
    return launch_push<double>(static_cast<double*>(s->x), static_cast<double*>(s->v),
                               static_cast<const double*>(s->Ei), p.N, p.dt, p.L, s->s);
  return launch_push<float>(static_cast<float*>(s->x), static_cast<float*>(s->v), static_cast<const float*>(s->Ei),
                            p.N, p.dt, p.L, s->s);
}

// The fixed part of a step, the same launches with the same arguments every
// step. Standard PIC (linear weighting both ways, no width update): the
// whole step. KDE: deposit with kappa_i, field, energy, gather, push and
// the A^2 statistic. Both end with the copy of the mailbox (A^2, status)
// to the host.
static kde_status enqueue_fixed(kde_session* s) {
  const kde_pic_params& p = s->prm;
  if (standard(p)) {
    const double dx = p.L / double(p.M);
    KDE_RETURN_IF(deposit(&s->tdom, p.N, s->x, nullptr, dx, s->rho, s->ws, s->ws_bytes, s->s, status_word(s)));
    KDE_RETURN_IF(launch_poisson_field(s->rho, p.M, p.L, s->E, s->s));
    KDE_RETURN_IF(record_energy(s));
    KDE_RETURN_IF(gather(&s->tdom, p.N, s->x, nullptr, dx, s->E, s->Ei, s->s, status_word(s)));
    KDE_RETURN_IF(push_any(s));
  } else {
    KDE_RETURN_IF(deposit(&s->dom, p.N, s->x, s->kap, 0.0, s->rho, s->ws, s->ws_bytes, s->s, status_word(s)));
    KDE_RETURN_IF(launch_poisson_field(s->rho, p.M, p.L, s->E, s->s));
    KDE_RETURN_IF(record_energy(s));
    KDE_RETURN_IF(gather(&s->dom, p.N, s->x, s->kap, 0.0, s->E, s->Ei, s->s, status_word(s)));
    KDE_RETURN_IF(push_any(s));
    if (p.prec == KDE_F64)
      KDE_RETURN_IF(launch_ad_statistic<double>(static_cast<const double*>(s->x), p.N, p.L, &s->dmail->a2, s->ws,
                                                s->ws_bytes, s->s));
    else
      KDE_RETURN_IF(launch_ad_statistic<float>(static_cast<const float*>(s->x), p.N, p.L, &s->dmail->a2, s->ws,
                                               s->ws_bytes, s->s));
  }
  KDE_TRY_HIP(hipMemcpyAsync(s->mail, s->dmail, sizeof(SessionMail), hipMemcpyDeviceToHost, s->s));
  return KDE_OK;
}

// Enqueue the fixed part: captured into a graph at the first step (all its
// pointers are the session's own and its launch shapes depend on N and M
// alone), then one graph launch per step instead of some twenty kernel
// launches.
static kde_status run_fixed(kde_session* s) {
  if (!s->fixed) {
    KDE_TRY_HIP(hipStreamBeginCapture(s->s, hipStreamCaptureModeRelaxed));
    const kde_status st = enqueue_fixed(s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s->s, &g);
    if (st != KDE_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    KDE_TRY_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&s->fixed, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      s->fixed = nullptr;
      KDE_TRY_HIP(ei);
    }
  }
  KDE_TRY_HIP(hipGraphLaunch(s->fixed, s->s));
  return KDE_OK;
}

static kde_status numeric_failure(kde_session* s) {
  return fail(KDE_E_NUMERIC, "session met non-finite %s%s%s (step %lld)",
              (s->numeric & KDE_NUMERIC_POSITION) ? "positions" : "",
              (s->numeric & KDE_NUMERIC_POSITION) && (s->numeric & KDE_NUMERIC_CONCENTRATION) ? " and " : "",
              (s->numeric & KDE_NUMERIC_CONCENTRATION) ? "concentrations" : (s->numeric ? "" : "values"),
              (long long)s->st.step);
}

// The end of a step: relax the width, enqueue the next widths.
static kde_status finish_step(kde_session* s) {
  const kde_pic_params& p = s->prm;
  SessionState& st = s->st;
  st.h_opt = p.adjust_rate * st.h_target + (1.0 - p.adjust_rate) * st.h_opt;
  st.kappa_star = kappa_of_width(st.h_opt, p.L);
  KDE_RETURN_IF(session_widths(s, st.kappa_star));
  st.step += 1;
  s->phase = StepPhase::Idle;
  return KDE_OK;
}

kde_status session_begin_step(kde_session* s) {
  if (s->phase != StepPhase::Idle) return fail(KDE_E_INTERNAL, "a step of this session is in flight");
  s->t_begin = std::chrono::steady_clock::now();
  KDE_RETURN_IF(run_fixed(s));
  KDE_TRY_HIP(hipEventRecord(s->ev, s->s));
  s->phase = StepPhase::Fixed;
  return KDE_OK;
}

kde_status session_advance(kde_session* s, bool* done) {
  *done = false;
  const kde_pic_params& p = s->prm;
  SessionState& st = s->st;
  if (s->phase == StepPhase::Fixed) {
    s->numeric |= s->mail->status;
    if (standard(p)) {
      st.step += 1;
      s->phase = StepPhase::Idle;
      *done = true;
      return s->numeric ? numeric_failure(s) : KDE_OK;
    }
    st.last_a2 = s->mail->a2;
    // A^2 of positions in [0, L) (logs clamped) is finite: a non-finite one
    // means the push produced a non-finite position
    if (!std::isfinite(st.last_a2)) s->numeric |= KDE_NUMERIC_POSITION;
    if (s->numeric) {
      // a non-finite position or width reached the step: the rule and the
      // widths are left as they were, the step is counted
      st.step += 1;
      s->phase = StepPhase::Idle;
      *done = true;
      return numeric_failure(s);
    }
    st.last_p = ad_upper_tail(st.last_a2);
    const double thr = p.p_threshold;
    if (st.last_p > 2.0 * thr) {
      st.p_th = 2.0 * thr;
    } else if (st.last_p < 0.5 * st.p_th) {
      KDE_RETURN_IF(enqueue_cv(s));
      KDE_TRY_HIP(hipEventRecord(s->ev, s->s));
      s->phase = StepPhase::Scan;
      return KDE_OK;
    }
    KDE_RETURN_IF(finish_step(s));
    *done = true;
    return KDE_OK;
  }
  if (s->phase == StepPhase::Scan) {
    s->numeric |= s->mail->status;
    double k = 0.0;
    KDE_RETURN_IF(scanned_kappa(s, &k));
    st.h_target = width_of_kappa(k, p.L);
    st.p_th = st.last_p;
    st.fired += 1;
    KDE_RETURN_IF(finish_step(s));
    *done = true;
    return KDE_OK;
  }
  return fail(KDE_E_INTERNAL, "no step of this session is in flight");
}

hipEvent_t session_event(const kde_session* s) { return s->ev; }
size_t session_arena_bytes(const kde_session* s) { return s->arena_bytes; }
double session_step_seconds(const kde_session* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t_begin).count();
}

// One step on the calling thread, waiting on the session's event.
static kde_status session_step_once(kde_session* s) {
  KDE_RETURN_IF(session_begin_step(s));
  bool done = false;
  while (!done) {
    KDE_TRY_HIP(hipEventSynchronize(s->ev));
    KDE_RETURN_IF(session_advance(s, &done));
  }
  return KDE_OK;
}

}  // namespace kde

extern "C" {

kde_status kde_ad_pvalue(double a2, double* p_h) {
  clear_error();
  if (!p_h) return fail(KDE_E_INVALID_ARG, "p_h is NULL");
  *p_h = ad_upper_tail(a2);
  return KDE_OK;
}

kde_status kde_session_bytes(const kde_pic_params* p, size_t* bytes_h) {
  clear_error();
  KDE_RETURN_IF(check_params(p));
  if (!bytes_h) return fail(KDE_E_INVALID_ARG, "bytes_h is NULL");
  Carver c(nullptr, 0);
  *bytes_h = carve_session(c, *p, nullptr);
  return KDE_OK;
}

kde_status kde_session_create(const kde_pic_params* p, const void* x0, const void* v0, void* arena, size_t arena_bytes,
                              void* stream, kde_session** out_h) {
  clear_error();
  if (!out_h) return fail(KDE_E_INVALID_ARG, "out_h is NULL");
  *out_h = nullptr;
  KDE_RETURN_IF(check_params(p));
  if (!x0 || !v0) return fail(KDE_E_INVALID_ARG, "x0 and v0 must not be NULL");
  std::unique_ptr<kde_session> s(new kde_session());
  s->prm = *p;
  if (!standard(*p)) s->kappas.assign(p->kappas_h, p->kappas_h + p->B);
  s->prm.kappas_h = nullptr;
  s->dom = kde_domain{p->L, p->M, p->prec, KDE_SHAPE_VONMISES, 0};
  s->tdom = kde_domain{p->L, p->M, p->prec, KDE_SHAPE_TRIANGLE, 0};
  Carver c(arena, arena_bytes);
  carve_session(c, *p, s.get());
  if (!arena || reinterpret_cast<uintptr_t>(arena) % 256 != 0) return fail(KDE_E_WORKSPACE, "arena must be 256-byte aligned");
  if (!c.fits()) return fail(KDE_E_WORKSPACE, "arena too small: %zu < %zu bytes", arena_bytes, c.used);
  s->arena_bytes = c.used;
  KDE_TRY_HIP(hipStreamCreateWithFlags(&s->s, hipStreamNonBlocking));
  KDE_TRY_HIP(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming));
  KDE_TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->mail), sizeof(SessionMail), hipHostMallocDefault));
  // the copies of x0 and v0 follow the work already enqueued on the caller's stream
  KDE_TRY_HIP(hipEventRecord(s->ev, static_cast<hipStream_t>(stream)));
  KDE_TRY_HIP(hipStreamWaitEvent(s->s, s->ev, 0));
  const size_t es = elem_size(p->prec);
  KDE_TRY_HIP(hipMemcpyAsync(s->x, x0, size_t(p->N) * es, hipMemcpyDeviceToDevice, s->s));
  KDE_TRY_HIP(hipMemcpyAsync(s->v, v0, size_t(p->N) * es, hipMemcpyDeviceToDevice, s->s));
  KDE_RETURN_IF(launch_set_step(s->step_dev, 0, s->s));
  KDE_RETURN_IF(clear_status(s.get()));
  if (standard(*p)) {
    KDE_TRY_HIP(hipStreamSynchronize(s->s));
    *out_h = s.release();
    return KDE_OK;
  }
  // initial CV at t = 0: both widths at its optimum, p_th = 2 thr
  KDE_RETURN_IF(enqueue_cv(s.get()));
  KDE_TRY_HIP(hipStreamSynchronize(s->s));
  if (s->mail->status) {
    s->numeric = s->mail->status;
    return numeric_failure(s.get());
  }
  double k0 = 0.0;
  KDE_RETURN_IF(scanned_kappa(s.get(), &k0));
  s->st.p_th = 2.0 * p->p_threshold;
  s->st.h_opt = s->st.h_target = width_of_kappa(k0, p->L);
  s->st.kappa_star = k0;
  KDE_RETURN_IF(session_widths(s.get(), k0));
  KDE_TRY_HIP(hipStreamSynchronize(s->s));
  *out_h = s.release();
  return KDE_OK;
}

kde_status kde_session_step(kde_session* s, int32_t nsteps) {
  clear_error();
  if (!s) return fail(KDE_E_NOT_FOUND, "session is NULL");
  if (nsteps < 0) return fail(KDE_E_INVALID_ARG, "nsteps must be >= 0");
  if (s->phase != StepPhase::Idle) return fail(KDE_E_INVALID_ARG, "a step of this session is in flight (attached to a server?)");
  if (standard(s->prm)) {  // enqueue only: standard steps never wait on the host
    for (int k = 0; k < nsteps; ++k) {
      KDE_RETURN_IF(run_fixed(s));
      s->st.step += 1;
    }
    KDE_TRY_HIP(hipStreamSynchronize(s->s));
    s->numeric |= s->mail->status;
    return s->numeric ? numeric_failure(s) : KDE_OK;
  }
  for (int k = 0; k < nsteps; ++k) KDE_RETURN_IF(session_step_once(s));
  KDE_TRY_HIP(hipStreamSynchronize(s->s));
  return KDE_OK;
}

kde_status kde_session_state(const kde_session* s, kde_session_info* h) {
  clear_error();
  if (!s || !h) return fail(KDE_E_INVALID_ARG, "session and output must not be NULL");
  h->step = s->st.step;
  h->p_th = s->st.p_th;
  h->h_opt = s->st.h_opt;
  h->h_target = s->st.h_target;
  h->kappa_star = s->st.kappa_star;
  h->last_a2 = s->st.last_a2;
  h->last_p = s->st.last_p;
  h->fired = s->st.fired;
  h->numeric = s->numeric;
  h->reserved = 0;
  return KDE_OK;
}

kde_status kde_session_read(kde_session* s, int32_t what, void* dst) {
  clear_error();
  if (!s || !dst) return fail(KDE_E_INVALID_ARG, "session and dst must not be NULL");
  const size_t pn = size_t(s->prm.N) * elem_size(s->prm.prec), gm = size_t(s->prm.M) * sizeof(double);
  const void* src = nullptr;
  size_t bytes = 0;
  switch (what) {
    case KDE_SESSION_X: src = s->x; bytes = pn; break;
    case KDE_SESSION_V: src = s->v; bytes = pn; break;
    case KDE_SESSION_KAPPA: src = s->kap; bytes = pn; break;
    case KDE_SESSION_RHO: src = s->rho; bytes = gm; break;
    case KDE_SESSION_E: src = s->E; bytes = gm; break;
    case KDE_SESSION_ENERGY:
      src = s->energy;
      bytes = size_t(std::min<int64_t>(s->st.step, s->prm.history)) * sizeof(double);
      break;
    default: return fail(KDE_E_INVALID_ARG, "unknown field %d", what);
  }
  if (bytes == 0) return KDE_OK;
  KDE_TRY_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s->s));
  KDE_TRY_HIP(hipStreamSynchronize(s->s));
  return KDE_OK;
}

// Blob: magic, header (N, M, prec, method, history), state, then x, v,
// kappa_i and the energy history.
static const uint64_t kMagic = 0x6b64657069637332ull;  // "kdepics2"

static size_t blob_bytes(const kde_session* s) {
  const size_t pn = size_t(s->prm.N) * elem_size(s->prm.prec);
  return 64 + sizeof(SessionState) + 3 * pn + size_t(s->prm.history) * sizeof(double);
}

kde_status kde_session_save(kde_session* s, void* blob_h, size_t* bytes_h) {
  clear_error();
  if (!s || !bytes_h) return fail(KDE_E_INVALID_ARG, "session and bytes_h must not be NULL");
  const size_t pn = size_t(s->prm.N) * elem_size(s->prm.prec);
  const size_t need = blob_bytes(s);
  if (!blob_h) {
    *bytes_h = need;
    return KDE_OK;
  }
  if (*bytes_h < need) return fail(KDE_E_INVALID_ARG, "blob too small: %zu < %zu", *bytes_h, need);
  char* b = static_cast<char*>(blob_h);
  memset(b, 0, 64);
  memcpy(b, &kMagic, 8);
  const int64_t hdr[5] = {s->prm.N, s->prm.M, s->prm.prec, s->prm.method, s->prm.history};
  memcpy(b + 8, hdr, sizeof hdr);
  memcpy(b + 64, &s->st, sizeof(SessionState));
  char* p = b + 64 + sizeof(SessionState);
  KDE_TRY_HIP(hipMemcpyAsync(p, s->x, pn, hipMemcpyDeviceToHost, s->s));
  KDE_TRY_HIP(hipMemcpyAsync(p + pn, s->v, pn, hipMemcpyDeviceToHost, s->s));
  KDE_TRY_HIP(hipMemcpyAsync(p + 2 * pn, s->kap, pn, hipMemcpyDeviceToHost, s->s));
  if (s->prm.history > 0)
    KDE_TRY_HIP(hipMemcpyAsync(p + 3 * pn, s->energy, size_t(s->prm.history) * sizeof(double), hipMemcpyDeviceToHost,
                               s->s));
  KDE_TRY_HIP(hipStreamSynchronize(s->s));
  *bytes_h = need;
  return KDE_OK;
}

kde_status kde_session_restore(kde_session* s, const void* blob_h, size_t bytes) {
  clear_error();
  if (!s || !blob_h) return fail(KDE_E_INVALID_ARG, "session and blob must not be NULL");
  if (s->phase != StepPhase::Idle) return fail(KDE_E_INVALID_ARG, "a step of this session is in flight");
  const size_t pn = size_t(s->prm.N) * elem_size(s->prm.prec);
  const size_t need = blob_bytes(s);
  if (bytes < need) return fail(KDE_E_INVALID_ARG, "blob too small: %zu < %zu", bytes, need);
  const char* b = static_cast<const char*>(blob_h);
  uint64_t magic = 0;
  int64_t hdr[5];
  memcpy(&magic, b, 8);
  memcpy(hdr, b + 8, sizeof hdr);
  if (magic != kMagic || hdr[0] != s->prm.N || hdr[1] != s->prm.M || hdr[2] != s->prm.prec ||
      hdr[3] != s->prm.method || hdr[4] != s->prm.history)
    return fail(KDE_E_INVALID_ARG, "blob does not belong to a session of this shape");
  memcpy(&s->st, b + 64, sizeof(SessionState));
  const char* p = b + 64 + sizeof(SessionState);
  KDE_TRY_HIP(hipMemcpyAsync(s->x, p, pn, hipMemcpyHostToDevice, s->s));
  KDE_TRY_HIP(hipMemcpyAsync(s->v, p + pn, pn, hipMemcpyHostToDevice, s->s));
  KDE_TRY_HIP(hipMemcpyAsync(s->kap, p + 2 * pn, pn, hipMemcpyHostToDevice, s->s));
  if (s->prm.history > 0)
    KDE_TRY_HIP(hipMemcpyAsync(s->energy, p + 3 * pn, size_t(s->prm.history) * sizeof(double), hipMemcpyHostToDevice,
                               s->s));
  KDE_RETURN_IF(launch_set_step(s->step_dev, s->st.step, s->s));
  KDE_RETURN_IF(clear_status(s));
  s->numeric = 0;
  KDE_TRY_HIP(hipStreamSynchronize(s->s));
  return KDE_OK;
}

kde_status kde_damping_rate(const double* energy_h, int64_t n, double dt, double* rate_h, int64_t* peaks_h) {
  clear_error();
  if (!energy_h || !rate_h) return fail(KDE_E_INVALID_ARG, "energy_h and rate_h must not be NULL");
  if (n < 3) return fail(KDE_E_INVALID_ARG, "need at least 3 energies (got %lld)", (long long)n);
  if (!std::isfinite(dt) || !(dt > 0.0)) return fail(KDE_E_INVALID_ARG, "dt must be finite and > 0");
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(energy_h[k]) || !(energy_h[k] > 0.0))
      return fail(KDE_E_INVALID_ARG, "energies must be finite and > 0 (index %lld)", (long long)k);
  int64_t pk[2] = {-1, -1};
  int found = 0;
  for (int64_t k = 1; k + 1 < n && found < 2; ++k)
    if (energy_h[k - 1] < energy_h[k] && energy_h[k] >= energy_h[k + 1]) pk[found++] = k;
  if (peaks_h) {
    peaks_h[0] = pk[0];
    peaks_h[1] = pk[1];
  }
  *rate_h = (found < 2) ? std::nan("")
                        : (std::log(energy_h[pk[1]]) - std::log(energy_h[pk[0]])) / (double(pk[1] - pk[0]) * dt);
  return KDE_OK;
}

kde_status kde_session_destroy(kde_session* s) {
  clear_error();
  if (s) {
    if (s->s) {
      (void)hipStreamSynchronize(s->s);
      (void)hipStreamDestroy(s->s);
    }
    delete s;
  }
  return KDE_OK;
}

}  // extern "C"
