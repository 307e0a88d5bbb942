// Request server (serving form): continuous batching of KDE solves beside
// resident PIC sessions.
//
// A request is one particle set taken through the whole path (CV scan on
// its first n_cv particles, pilot deposit at kappa*, adaptive widths,
// adaptive deposit), exactly as one set of a batch. The scheduling policy
// (sched.hpp) decides what runs when; this file is its device side: slots
// (a HIP stream of default priority, a completion event and pinned staging
// each) run groups of requests through the batched engine with one
// workgroup per work unit, so slots and the sessions' own streams share the
// compute units as workgroups retire. A scheduler thread advances the slots
// and the attached sessions (each session step is a state machine driven by
// event queries, so the thread never waits on the device) and admits
// queued requests as slots and arena space free up. Every request waits for
// the work its submitter had enqueued on its own stream (an event recorded
// at submission). A set's results do not depend on the other sets of its
// group, so every request gets the same bits alone or in any mix. Latency is
// completion (the scheduler noticing the slot's event) minus submission, on
// the host's steady clock.
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_internal.hpp"
#include "sched.hpp"
#include "session_internal.hpp"

namespace kde {

using sched::Clock;

// Estimated work of a request in term evaluations: the CV pair sums, the
// two deposits, and a fixed per-request overhead of about as many terms as
// the device evaluates in 20 microseconds.
static double request_cost(const kde_batch_set& e, int B) {
  const double ncv = double(e.n_cv);
  return double(B) * ncv * (ncv - 1.0) / 2.0 + 2.0 * double(e.N) * double(e.M) + 5.0e7;
}

constexpr size_t kStagingBytes = size_t(1) << 20;

struct SlotHw {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* staging = nullptr;
  BatchPlan plan;
};

struct RequestRec {
  kde_batch_set set;
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream
};

class HipExecutor : public sched::Executor {
 public:
  HipExecutor(const kde_server_config& cfg, const std::vector<double>& kappas, char* arena)
      : cfg_(cfg), kappas_(kappas), arena_(arena) {}
  ~HipExecutor() override {
    for (auto& kv : reqs_)
      if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    for (SlotHw& h : hw_) {
      if (h.stream) {
        (void)hipStreamSynchronize(h.stream);
        (void)hipStreamDestroy(h.stream);
      }
      if (h.done) (void)hipEventDestroy(h.done);
      if (h.staging) (void)hipHostFree(h.staging);
    }
  }

  kde_status init(int nslots) {
    hw_.resize(size_t(nslots));
    for (SlotHw& h : hw_) {
      KDE_TRY_HIP(hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
      KDE_TRY_HIP(hipEventCreateWithFlags(&h.done, hipEventDisableTiming));
      KDE_TRY_HIP(hipHostMalloc(&h.staging, kStagingBytes, hipHostMallocDefault));
    }
    return KDE_OK;
  }

  void add_request(uint64_t t, const kde_batch_set& e, hipEvent_t ready) { reqs_[t] = RequestRec{e, ready}; }
  void add_session(uint64_t t, kde_session* s) { sess_[t] = s; }

  kde_status plan_of(const std::vector<uint64_t>& tickets, BatchPlan& p) {
    std::vector<kde_batch_set> sets;
    sets.reserve(tickets.size());
    for (uint64_t t : tickets) sets.push_back(reqs_.at(t).set);
    KDE_RETURN_IF(batch_plan_make(sets.data(), int(sets.size()), cfg_.prec, cfg_.B, kappas_.data(), cfg_.alpha, p));
    p.resident_grids = false;
    if (batch_staging_bytes(p) > kStagingBytes) return fail(KDE_E_INTERNAL, "group descriptors exceed the staging");
    return KDE_OK;
  }

  bool group_bytes(const std::vector<uint64_t>& tickets, size_t* bytes) override {
    BatchPlan p;
    if (plan_of(tickets, p) != KDE_OK) return false;
    *bytes = p.ws_need;
    return true;
  }

  kde_status launch(int slot, const std::vector<uint64_t>& tickets, size_t off) override {
    SlotHw& h = hw_[size_t(slot)];
    KDE_RETURN_IF(plan_of(tickets, h.plan));
    for (uint64_t t : tickets) {
      const hipEvent_t ready = reqs_.at(t).ready;
      if (ready) KDE_TRY_HIP(hipStreamWaitEvent(h.stream, ready, 0));
    }
    KDE_RETURN_IF(batch_plan_enqueue(h.plan, arena_ + off, h.stream, h.staging));
    KDE_TRY_HIP(hipEventRecord(h.done, h.stream));
    return KDE_OK;
  }

  kde_status poll(int slot) override {
    const hipError_t q = hipEventQuery(hw_[size_t(slot)].done);
    if (q == hipSuccess) return KDE_OK;
    if (q == hipErrorNotReady) return KDE_E_AGAIN;
    return fail(KDE_E_HIP, "request work failed: %s", hipGetErrorString(q));
  }

  void outcomes(int slot, std::vector<kde_status>* st) override {
    const SlotHw& h = hw_[size_t(slot)];
    const uint32_t* w = batch_staged_status(h.plan, h.staging);
    st->clear();
    for (size_t k = 0; k < h.plan.sets.size(); ++k) st->push_back(w[k] ? KDE_E_NUMERIC : KDE_OK);
  }

  void forget(uint64_t t) override {
    auto it = reqs_.find(t);
    if (it != reqs_.end()) {
      if (it->second.ready) (void)hipEventDestroy(it->second.ready);
      reqs_.erase(it);
    }
    sess_.erase(t);
  }

  kde_status session_begin(uint64_t t) override { return session_begin_step(sess_.at(t)); }

  kde_status session_poll(uint64_t t) override {
    const hipError_t q = hipEventQuery(session_event(sess_.at(t)));
    if (q == hipSuccess) return KDE_OK;
    if (q == hipErrorNotReady) return KDE_E_AGAIN;
    return fail(KDE_E_HIP, "session step failed: %s", hipGetErrorString(q));
  }

  kde_status session_advance(uint64_t t, bool* done) override { return kde::session_advance(sess_.at(t), done); }

 private:
  kde_server_config cfg_;
  std::vector<double> kappas_;
  char* arena_;
  std::vector<SlotHw> hw_;
  std::unordered_map<uint64_t, RequestRec> reqs_;
  std::unordered_map<uint64_t, kde_session*> sess_;
};

}  // namespace kde

using namespace kde;

struct kde_server {
  kde_server_config cfg{};
  int device = 0;
  std::vector<double> kappas;
  std::unique_ptr<HipExecutor> ex;
  std::unique_ptr<sched::Scheduler> sch;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::atomic<bool> stop{false};
  std::thread worker;
};

namespace kde {

static kde_batch_set effective(const kde_server* s, const kde_batch_set& r) {
  kde_batch_set e = r;
  int64_t cap = s->cfg.n_cv > 0 ? s->cfg.n_cv : r.N;
  if (r.n_cv > 0) cap = std::min(cap, r.n_cv);
  e.n_cv = std::min<int64_t>(cap, r.N);
  return e;
}

static void worker_loop(kde_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    const bool busy = s->sch->tick(Clock::now());
    s->cv_done.notify_all();
    if (busy)
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else
      s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

}  // namespace kde

extern "C" {

kde_status kde_server_create(const kde_server_config* cfg, void* arena, size_t budget_bytes, kde_server** out_h) {
  clear_error();
  if (!out_h || !cfg) return fail(KDE_E_INVALID_ARG, "config and out_h must not be NULL");
  *out_h = nullptr;
  if (cfg->prec != KDE_F64 && cfg->prec != KDE_F32) return fail(KDE_E_INVALID_ARG, "prec must be KDE_F64 or KDE_F32");
  if (cfg->B < 1 || cfg->B > KDE_MAX_KAPPAS || !cfg->kappas_h) return fail(KDE_E_INVALID_ARG, "B must lie in [1, 64]");
  for (int b = 0; b < cfg->B; ++b)
    if (!std::isfinite(cfg->kappas_h[b]) || cfg->kappas_h[b] < 0.0 || cfg->kappas_h[b] > KDE_MAX_CV_KAPPA ||
        (b > 0 && !(cfg->kappas_h[b] > cfg->kappas_h[b - 1])))
      return fail(KDE_E_INVALID_ARG, "kappas must lie in [0, %g] and be strictly ascending", KDE_MAX_CV_KAPPA);
  if (cfg->nslots < 1 || cfg->nslots > 64) return fail(KDE_E_INVALID_ARG, "nslots must lie in [1, 64]");
  if (cfg->max_batch < 1 || cfg->max_batch > 1024) return fail(KDE_E_INVALID_ARG, "max_batch must lie in [1, 1024]");
  if (!std::isfinite(cfg->alpha) || cfg->alpha < 0.0) return fail(KDE_E_INVALID_ARG, "alpha must be finite and >= 0");
  if (cfg->large_slots < 0 || !(cfg->large_terms >= 0.0) || !std::isfinite(cfg->large_terms))
    return fail(KDE_E_INVALID_ARG, "large_slots and large_terms must be >= 0 (0 = default)");
  if (!arena || reinterpret_cast<uintptr_t>(arena) % 256 != 0 || budget_bytes < 256)
    return fail(KDE_E_WORKSPACE, "arena must be 256-byte aligned and hold at least 256 bytes");
  std::unique_ptr<kde_server> s(new kde_server());
  s->cfg = *cfg;
  s->kappas.assign(cfg->kappas_h, cfg->kappas_h + cfg->B);
  s->cfg.kappas_h = nullptr;
  KDE_TRY_HIP(hipGetDevice(&s->device));
  s->ex.reset(new HipExecutor(s->cfg, s->kappas, static_cast<char*>(arena)));
  KDE_RETURN_IF(s->ex->init(cfg->nslots));
  sched::Config sc;
  sc.nslots = cfg->nslots;
  sc.max_batch = cfg->max_batch;
  sc.large_slots = cfg->large_slots > 0 ? std::min(cfg->large_slots, cfg->nslots) : 1;
  sc.large_terms = cfg->large_terms > 0.0 ? cfg->large_terms : 2.0e9;
  sc.budget = budget_bytes;
  s->sch.reset(new sched::Scheduler(sc, s->ex.get()));
  kde_server* raw = s.get();
  s->worker = std::thread(worker_loop, raw);
  *out_h = s.release();
  return KDE_OK;
}

kde_status kde_server_request_bytes(const kde_server* s, const kde_batch_set* req_h, size_t* bytes_h) {
  clear_error();
  if (!s || !req_h || !bytes_h) return fail(KDE_E_INVALID_ARG, "server, request and bytes_h must not be NULL");
  const kde_batch_set e = effective(s, *req_h);
  BatchPlan p;
  KDE_RETURN_IF(batch_plan_make(&e, 1, s->cfg.prec, s->cfg.B, s->kappas.data(), s->cfg.alpha, p));
  *bytes_h = p.ws_need;
  return KDE_OK;
}

kde_status kde_server_submit(kde_server* s, const kde_batch_set* req_h, void* stream, uint64_t* ticket_h) {
  clear_error();
  if (!s || !req_h || !ticket_h) return fail(KDE_E_INVALID_ARG, "server, request and ticket_h must not be NULL");
  const kde_batch_set e = effective(s, *req_h);
  BatchPlan p;
  KDE_RETURN_IF(batch_plan_make(&e, 1, s->cfg.prec, s->cfg.B, s->kappas.data(), s->cfg.alpha, p));
  hipEvent_t ready = nullptr;
  KDE_TRY_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  const hipError_t er = hipEventRecord(ready, static_cast<hipStream_t>(stream));
  if (er != hipSuccess) {
    (void)hipEventDestroy(ready);
    return fail(KDE_E_HIP, "recording the submitter's stream failed: %s", hipGetErrorString(er));
  }
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t t = s->sch->new_ticket();
  const double ncv = double(e.n_cv);
  const kde_status st = s->sch->submit(t, request_cost(e, s->cfg.B), p.ws_need, Clock::now(),
                                       double(s->cfg.B) * ncv * (ncv - 1.0) / 2.0, double(e.N));
  if (st != KDE_OK) {
    (void)hipEventDestroy(ready);
    return fail(st, "request needs %zu bytes, more than the whole budget", p.ws_need);
  }
  s->ex->add_request(t, e, ready);
  *ticket_h = t;
  s->cv_work.notify_one();
  return KDE_OK;
}

kde_status kde_server_attach(kde_server* s, kde_session* session, int64_t nsteps, uint64_t* ticket_h) {
  clear_error();
  if (!s || !session || !ticket_h) return fail(KDE_E_INVALID_ARG, "server, session and ticket_h must not be NULL");
  if (nsteps < 0) return fail(KDE_E_INVALID_ARG, "nsteps must be >= 0");
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t t = s->sch->new_ticket();
  const size_t bytes = session_arena_bytes(session);
  const kde_status st = s->sch->attach(t, bytes, nsteps, Clock::now());
  if (st != KDE_OK) return fail(st, "session arena of %zu bytes does not fit in the free budget", bytes);
  s->ex->add_session(t, session);
  *ticket_h = t;
  s->cv_work.notify_one();
  return KDE_OK;
}

kde_status kde_server_cancel(kde_server* s, uint64_t ticket) {
  clear_error();
  if (!s) return fail(KDE_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  const kde_status st = s->sch->cancel(ticket, Clock::now());
  if (st == KDE_E_NOT_FOUND) return fail(st, "ticket %llu is neither queued nor attached", (unsigned long long)ticket);
  if (st == KDE_E_AGAIN) return KDE_E_AGAIN;
  s->cv_done.notify_all();
  return st;
}

// Fills res_h from a completed ticket's outcome; returns its status.
static kde_status report(uint64_t ticket, const sched::Outcome& o, kde_result* res_h) {
  memset(res_h, 0, sizeof *res_h);
  res_h->status = o.status;
  res_h->batch_size = o.batch_size;
  res_h->latency_s = o.latency_s;
  res_h->queue_s = o.queue_s;
  res_h->run_s = o.run_s;
  res_h->steps = o.steps;
  if (o.status != KDE_OK) return fail(o.status, "ticket %llu ended with %s", (unsigned long long)ticket, kde_status_str(o.status));
  return KDE_OK;
}

kde_status kde_server_poll(kde_server* s, uint64_t ticket, kde_result* res_h) {
  clear_error();
  if (!s || !res_h) return fail(KDE_E_INVALID_ARG, "server and res_h must not be NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  sched::Outcome o;
  const kde_status st = s->sch->poll(ticket, &o);
  if (st == KDE_E_NOT_FOUND) return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
  if (st == KDE_E_AGAIN) return KDE_E_AGAIN;
  return report(ticket, o, res_h);
}

kde_status kde_server_wait(kde_server* s, uint64_t ticket, kde_result* res_h) {
  clear_error();
  if (!s || !res_h) return fail(KDE_E_INVALID_ARG, "server and res_h must not be NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  sched::Outcome o;
  kde_status st = s->sch->poll(ticket, &o);
  if (st == KDE_E_NOT_FOUND) return fail(st, "unknown ticket %llu", (unsigned long long)ticket);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [&] {
    st = s->sch->poll(ticket, &o);
    return st != KDE_E_AGAIN;
  });
  return report(ticket, o, res_h);
}

kde_status kde_server_drain(kde_server* s) {
  clear_error();
  if (!s) return fail(KDE_E_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [&] { return !s->sch->busy(); });
  return KDE_OK;
}

kde_status kde_server_stats(kde_server* s, kde_server_stats_t* st) {
  clear_error();
  if (!s || !st) return fail(KDE_E_INVALID_ARG, "server and st must not be NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  const sched::Stats& x = s->sch->stats();
  memset(st, 0, sizeof *st);
  st->submitted = x.submitted;
  st->completed = x.completed;
  st->rejected = x.rejected;
  st->launches = x.launches;
  st->mean_batch = x.launches ? double(x.batched) / double(x.launches) : 0.0;
  if (!x.latencies.empty()) {
    st->p50_s = sched::quantile(x.latencies, 0.50);
    st->p99_s = sched::quantile(x.latencies, 0.99);
    st->max_s = sched::quantile(x.latencies, 1.0);
    double sum = 0.0;
    for (double v : x.latencies) sum += v;
    st->mean_s = sum / double(x.latencies.size());
  }
  st->wall_s = x.have_first && (x.completed || x.session_steps) ? sched::seconds(x.first, x.last) : 0.0;
  st->requests_per_s = st->wall_s > 0 ? double(x.completed) / st->wall_s : 0.0;
  st->pair_evals = x.pair_evals;
  st->particles = x.particles;
  st->failed = x.failed;
  st->cancelled = x.cancelled;
  st->session_steps = x.session_steps;
  st->session_p50_s = sched::quantile(x.step_latencies, 0.50);
  st->session_p99_s = sched::quantile(x.step_latencies, 0.99);
  return KDE_OK;
}

kde_status kde_server_destroy(kde_server* s) {
  clear_error();
  if (!s) return KDE_OK;
  {
    // queued requests are dropped; running groups and the attached
    // sessions' steps in flight finish, so every session is left between
    // steps and can be stepped, saved or destroyed by its owner
    std::unique_lock<std::mutex> lk(s->mu);
    s->sch->close(Clock::now());
    s->cv_work.notify_one();
    s->cv_done.wait(lk, [&] { return !s->sch->busy(); });
    s->stop.store(true);
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->sch.reset();
  s->ex.reset();
  delete s;
  return KDE_OK;
}

}  // extern "C"
