// Request server (serving form): continuous batching of KDE solves.
//
// A request is one particle set taken through the whole path (CV scan on
// its first n_cv particles, pilot deposit at kappa*, adaptive widths,
// adaptive deposit), exactly as one set of a batch. Requests wait in a FIFO
// queue. A scheduler thread admits them into slots: a slot is a HIP stream
// (default priority) with a pinned staging buffer. Requests are large or
// small by estimated work. Large ones run alone, at most `large_slots` at
// a time, in arrival order: sharing the device among several large solves
// would stretch each of them, and they set the latency tail. When a slot is
// free and no large request may start, the oldest small request heads a
// new batch, joined by up to `max_batch - 1` later small requests of
// comparable cost (between a quarter and twice the head's estimated work,
// so that none waits on a much longer one inside a batch) whose workspaces
// fit together in the free part of the arena (first fit). The batch's phase
// kernels are enqueued on the slot's stream
// with one workgroup per work unit, so slots, and other streams such as
// resident PIC sessions, share the compute units as workgroups retire; then
// an event is recorded. Requests that arrive while others run are admitted
// as soon as a slot and arena space free up.
// A request larger than the whole budget is refused at submission. Because
// a set's results do not depend on the other sets of its batch, every
// request gets the same bits alone or in any mix. Latency is completion
// (the host noticing the slot's event) minus submission, on the host's
// steady clock.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_internal.hpp"

namespace kde {

using Clock = std::chrono::steady_clock;

static double seconds_since(Clock::time_point t0, Clock::time_point t) {
  return std::chrono::duration<double>(t - t0).count();
}

// First-fit allocator of 256-byte aligned blocks inside the arena.
class ArenaAlloc {
 public:
  void reset(size_t cap) {
    free_.clear();
    free_[0] = cap;
    cap_ = cap;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(bytes, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes, 256);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0;
};

struct Pending {
  uint64_t ticket;
  kde_batch_set req;
  Clock::time_point arrival;
  size_t alone_bytes;
  double cost;  // estimated work (request_cost)
};

// Estimated work of a request in term evaluations: the CV pair sums, the
// two deposits, and a fixed per-request overhead of about as many terms as
// the device evaluates in 20 microseconds.
static double request_cost(const kde_batch_set& e, int B) {
  const double ncv = double(e.n_cv);
  return double(B) * ncv * (ncv - 1.0) / 2.0 + 2.0 * double(e.N) * double(e.M) + 5.0e7;
}

static bool joins(double cost, double head) { return cost <= 2.0 * head && cost >= 0.25 * head; }

// Requests of the queue scanned for batch partners per admission.
constexpr size_t kAdmitScan = 256;

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* staging = nullptr;
  bool busy = false;
  bool large = false;  // running a large request
  size_t off = 0, bytes = 0;
  std::vector<Pending> reqs;
  Clock::time_point started;
};

constexpr size_t kStagingBytes = size_t(1) << 20;

}  // namespace kde

using namespace kde;

struct kde_server {
  kde_server_config cfg{};
  int device = 0;
  std::vector<double> kappas;
  char* arena = nullptr;
  size_t budget = 0;
  int large_slots = 1;
  double large_terms = 2.0e9;
  ArenaAlloc alloc;
  std::vector<Slot> slots;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, kde_result> results;
  std::vector<double> latencies;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, rejected = 0, launches = 0, batched_requests = 0;
  double pair_evals = 0.0, particles = 0.0;
  Clock::time_point t_first, t_last;
  bool have_first = false;
  kde_status fault = KDE_OK;
  char fault_msg[256] = {0};
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

static void finish_slot(kde_server* s, Slot& sl, Clock::time_point t) {
  for (const Pending& p : sl.reqs) {
    kde_result r{};
    r.status = KDE_OK;
    r.batch_size = int32_t(sl.reqs.size());
    r.latency_s = seconds_since(p.arrival, t);
    r.queue_s = seconds_since(p.arrival, sl.started);
    r.run_s = seconds_since(sl.started, t);
    s->results[p.ticket] = r;
    s->latencies.push_back(r.latency_s);
    s->completed += 1;
    const double ncv = double(p.req.n_cv);
    s->pair_evals += double(s->cfg.B) * ncv * (ncv - 1.0) / 2.0;
    s->particles += double(p.req.N);
  }
  s->t_last = t;
  s->alloc.release(sl.off, sl.bytes);
  sl.reqs.clear();
  sl.busy = false;
}

// Admit queued requests into free slots (lock held). A large request runs
// alone, and no more than `large_slots` of them at a time, oldest first; a
// small request may pass queued large ones and heads a batch of small
// partners of comparable cost. A head whose workspace does not fit waits
// (and so do the requests of its class behind it).
static void admit(kde_server* s) {
  for (Slot& sl : s->slots) {
    if (s->queue.empty()) return;
    if (sl.busy) continue;
    int large_running = 0;
    for (const Slot& o : s->slots) large_running += (o.busy && o.large) ? 1 : 0;
    const bool large_ok = large_running < s->large_slots;
    const size_t scan = std::min(s->queue.size(), kAdmitScan);
    size_t h = scan;
    for (size_t k = 0; k < scan; ++k) {
      const bool large = s->queue[k].cost >= s->large_terms;
      if (!large || large_ok) {
        h = k;
        break;
      }
    }
    if (h == scan) return;  // only large requests wait, and their slots are taken
    const bool head_large = s->queue[h].cost >= s->large_terms;
    const double head = s->queue[h].cost;
    const size_t room = s->alloc.largest();
    std::vector<Pending> group;
    std::vector<size_t> taken;
    std::vector<kde_batch_set> sets;
    BatchPlan plan;
    size_t off = 0;
    for (size_t k = h; k < scan && int(group.size()) < (head_large ? 1 : s->cfg.max_batch); ++k) {
      if (k > h && (s->queue[k].cost >= s->large_terms || !joins(s->queue[k].cost, head))) continue;
      sets.push_back(s->queue[k].req);
      BatchPlan trial;
      if (batch_plan_make(sets.data(), int(sets.size()), s->cfg.prec, s->cfg.B, s->kappas.data(), s->cfg.alpha,
                          trial) != KDE_OK ||
          trial.ws_need > room || batch_staging_bytes(trial) > kStagingBytes) {
        sets.pop_back();
        if (k == h) break;
        continue;
      }
      plan = std::move(trial);
      group.push_back(s->queue[k]);
      taken.push_back(k);
    }
    if (group.empty()) return;  // the head waits for arena space
    plan.resident_grids = false;
    if (!s->alloc.alloc(plan.ws_need, &off)) return;
    kde_status st = batch_plan_enqueue(plan, s->arena + off, sl.stream, sl.staging);
    hipError_t e = hipEventRecord(sl.done, sl.stream);
    if (st != KDE_OK || e != hipSuccess) {
      s->fault = st != KDE_OK ? st : KDE_E_HIP;
      snprintf(s->fault_msg, sizeof s->fault_msg, "%s", st != KDE_OK ? kde_last_error() : hipGetErrorString(e));
      s->alloc.release(off, plan.ws_need);
      return;
    }
    for (size_t k = taken.size(); k-- > 0;) s->queue.erase(s->queue.begin() + std::ptrdiff_t(taken[k]));
    sl.busy = true;
    sl.large = head_large;
    sl.off = off;
    sl.bytes = plan.ws_need;
    sl.reqs = std::move(group);
    sl.started = Clock::now();
    s->launches += 1;
    s->batched_requests += int64_t(sl.reqs.size());
  }
}

static void worker_loop(kde_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    bool any_busy = false;
    for (Slot& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipSuccess) {
        finish_slot(s, sl, Clock::now());
      } else if (q == hipErrorNotReady) {
        any_busy = true;
      } else {
        s->fault = KDE_E_HIP;
        snprintf(s->fault_msg, sizeof s->fault_msg, "%s", hipGetErrorString(q));
        finish_slot(s, sl, Clock::now());
      }
    }
    if (s->fault == KDE_OK) admit(s);
    for (Slot& sl : s->slots) any_busy = any_busy || sl.busy;
    s->cv_done.notify_all();
    if (any_busy)
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
  s->large_slots = cfg->large_slots > 0 ? std::min(cfg->large_slots, cfg->nslots) : 1;
  s->large_terms = cfg->large_terms > 0.0 ? cfg->large_terms : 2.0e9;
  s->kappas.assign(cfg->kappas_h, cfg->kappas_h + cfg->B);
  s->cfg.kappas_h = nullptr;
  s->arena = static_cast<char*>(arena);
  s->budget = budget_bytes;
  s->alloc.reset(budget_bytes);
  KDE_TRY_HIP(hipGetDevice(&s->device));
  s->slots.resize(cfg->nslots);
  for (Slot& sl : s->slots) {
    KDE_TRY_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    KDE_TRY_HIP(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    KDE_TRY_HIP(hipHostMalloc(&sl.staging, kStagingBytes, hipHostMallocDefault));
  }
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

kde_status kde_server_submit(kde_server* s, const kde_batch_set* req_h, uint64_t* ticket_h) {
  clear_error();
  if (!s || !req_h || !ticket_h) return fail(KDE_E_INVALID_ARG, "server, request and ticket_h must not be NULL");
  const kde_batch_set e = effective(s, *req_h);
  BatchPlan p;
  KDE_RETURN_IF(batch_plan_make(&e, 1, s->cfg.prec, s->cfg.B, s->kappas.data(), s->cfg.alpha, p));
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fault != KDE_OK) return fail(s->fault, "server stopped after an error: %s", s->fault_msg);
  if (p.ws_need > s->budget) {
    s->rejected += 1;
    return fail(KDE_E_BUDGET, "request needs %zu bytes, the whole budget is %zu", p.ws_need, s->budget);
  }
  const auto now = Clock::now();
  if (!s->have_first) {
    s->t_first = now;
    s->have_first = true;
  }
  Pending pe{s->next_ticket++, e, now, p.ws_need, request_cost(e, s->cfg.B)};
  s->queue.push_back(pe);
  s->submitted += 1;
  *ticket_h = pe.ticket;
  s->cv_work.notify_one();
  return KDE_OK;
}

kde_status kde_server_poll(kde_server* s, uint64_t ticket, kde_result* res_h) {
  clear_error();
  if (!s || !res_h) return fail(KDE_E_INVALID_ARG, "server and res_h must not be NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it != s->results.end()) {
    *res_h = it->second;
    return KDE_OK;
  }
  if (ticket == 0 || ticket >= s->next_ticket) return fail(KDE_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (s->fault != KDE_OK) return fail(s->fault, "server stopped after an error: %s", s->fault_msg);
  return KDE_E_AGAIN;
}

kde_status kde_server_drain(kde_server* s) {
  clear_error();
  if (!s) return fail(KDE_E_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [&] {
    if (s->fault != KDE_OK) return true;
    if (!s->queue.empty()) return false;
    for (const Slot& sl : s->slots)
      if (sl.busy) return false;
    return true;
  });
  if (s->fault != KDE_OK) return fail(s->fault, "server stopped after an error: %s", s->fault_msg);
  return KDE_OK;
}

kde_status kde_server_stats(kde_server* s, kde_server_stats_t* st) {
  clear_error();
  if (!s || !st) return fail(KDE_E_INVALID_ARG, "server and st must not be NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(st, 0, sizeof *st);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->launches = s->launches;
  st->mean_batch = s->launches ? double(s->batched_requests) / double(s->launches) : 0.0;
  std::vector<double> l = s->latencies;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto q = [&](double f) {
      const double pos = f * double(l.size() - 1);
      const size_t i = size_t(pos);
      const double t = pos - double(i);
      return i + 1 < l.size() ? l[i] * (1.0 - t) + l[i + 1] * t : l[i];
    };
    st->p50_s = q(0.50);
    st->p99_s = q(0.99);
    st->max_s = l.back();
    double sum = 0.0;
    for (double v : l) sum += v;
    st->mean_s = sum / double(l.size());
  }
  st->wall_s = s->have_first && s->completed ? seconds_since(s->t_first, s->t_last) : 0.0;
  st->requests_per_s = st->wall_s > 0 ? double(s->completed) / st->wall_s : 0.0;
  st->pair_evals = s->pair_evals;
  st->particles = s->particles;
  return KDE_OK;
}

kde_status kde_server_destroy(kde_server* s) {
  clear_error();
  if (!s) return KDE_OK;
  s->stop.store(true);
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Slot& sl : s->slots) {
    if (sl.stream) {
      (void)hipStreamSynchronize(sl.stream);
      (void)hipStreamDestroy(sl.stream);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.staging) (void)hipHostFree(sl.staging);
  }
  delete s;
  return KDE_OK;
}

}  // extern "C"
