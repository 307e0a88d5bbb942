// The request server's scheduler: queue, arena allocator, admission policy,
// results and statistics, and the stepping of attached PIC sessions. Host
// code only (no HIP): the device work goes through an Executor, which the
// server implements with HIP streams and events (server.hip) and host tests
// implement with a fake device. Not thread-safe by itself: the server calls
// every member with its mutex held.
//
// Requests are large or small by estimated work (cost). Large ones run
// alone, at most `large_slots` at a time, in arrival order. Otherwise the
// oldest small request heads a group, joined by up to max_batch - 1 later
// small requests whose cost lies within [1/4, 2] of the head's, whose
// workspaces fit together in the largest free block of the arena; small
// requests may pass waiting large ones. A head that does not fit waits.
// Attached sessions are charged their arena bytes while attached and are
// stepped one step in flight at a time, beside the slots; cancelling one
// detaches it after the step in flight. A failure is
// kept to the work it belongs to: a group whose launch or device work
// fails completes its own requests with that status and frees its slot; a
// session whose step fails completes its ticket with that status.
#pragma once

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/kde.h"

namespace kde {
namespace sched {

using Clock = std::chrono::steady_clock;

inline double seconds(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

inline size_t round256(size_t v) { return (v + 255) / 256 * 256; }

// First-fit allocator of 256-byte aligned blocks inside the arena.
class ArenaAlloc {
 public:
  void reset(size_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round256(bytes);
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
    bytes = round256(bytes);
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
  size_t total_free() const {
    size_t t = 0;
    for (auto& kv : free_) t += kv.second;
    return t;
  }

 private:
  std::map<size_t, size_t> free_;
};

// A queued request.
struct Request {
  uint64_t ticket;
  double cost;       // estimated work (terms)
  size_t bytes;      // workspace when run alone
  Clock::time_point arrival;
};

struct Outcome {
  kde_status status = KDE_OK;
  int32_t batch_size = 0;
  double latency_s = 0.0, queue_s = 0.0, run_s = 0.0;
  int64_t steps = 0;  // sessions: steps taken
};

// The device side of the scheduler.
class Executor {
 public:
  virtual ~Executor() = default;
  // Workspace bytes of these requests run as one group; false when they
  // cannot run together (the plan fails or its staging is too large).
  virtual bool group_bytes(const std::vector<uint64_t>& tickets, size_t* bytes) = 0;
  // Enqueue the group in `slot`, its workspace at arena offset `off`.
  virtual kde_status launch(int slot, const std::vector<uint64_t>& tickets, size_t off) = 0;
  // KDE_OK once the slot's work has completed, KDE_E_AGAIN while it runs,
  // another status if it failed.
  virtual kde_status poll(int slot) = 0;
  // After completion: the status of each request of the group (numeric).
  virtual void outcomes(int slot, std::vector<kde_status>* st) = 0;
  // The request's inputs are no longer referenced (done or cancelled).
  virtual void forget(uint64_t ticket) = 0;
  // Sessions: begin a step; poll its event (KDE_OK, KDE_E_AGAIN, error);
  // advance after the event (done when the step is complete).
  virtual kde_status session_begin(uint64_t ticket) = 0;
  virtual kde_status session_poll(uint64_t ticket) = 0;
  virtual kde_status session_advance(uint64_t ticket, bool* done) = 0;
};

struct Config {
  int nslots = 4;
  int max_batch = 16;
  int large_slots = 1;
  double large_terms = 2.0e9;
  size_t budget = 0;
  size_t scan = 256;  // queued requests scanned per admission
};

struct Stats {
  int64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, rejected = 0, launches = 0;
  int64_t batched = 0;
  double pair_evals = 0.0, particles = 0.0;
  std::vector<double> latencies, step_latencies;
  int64_t session_steps = 0;
  Clock::time_point first, last;
  bool have_first = false;
};

class Scheduler {
 public:
  struct Slot {
    bool busy = false, large = false;
    size_t off = 0, bytes = 0;
    std::vector<Request> reqs;
    Clock::time_point started;
  };
  struct Session {
    uint64_t ticket;
    size_t off, bytes;
    int64_t steps_left, steps_done = 0;
    bool in_flight = false, cancelled = false;
    Clock::time_point arrival, step_start;
  };

  Scheduler(const Config& c, Executor* ex) : cfg_(c), ex_(ex), slots_(size_t(c.nslots)) { alloc_.reset(c.budget); }

  uint64_t new_ticket() { return next_ticket_++; }
  bool known(uint64_t t) const { return t != 0 && t < next_ticket_; }

  // Queue a request; KDE_E_BUDGET when it alone needs more than the budget.
  kde_status submit(uint64_t ticket, double cost, size_t bytes, Clock::time_point now, double pair_evals,
                    double particles) {
    if (bytes > cfg_.budget) {
      stats_.rejected += 1;
      return KDE_E_BUDGET;
    }
    if (!stats_.have_first) {
      stats_.first = now;
      stats_.have_first = true;
    }
    queue_.push_back(Request{ticket, cost, bytes, now});
    work_[ticket] = {pair_evals, particles};
    stats_.submitted += 1;
    return KDE_OK;
  }

  // Charge a session's arena against the budget and step it `steps` times.
  kde_status attach(uint64_t ticket, size_t bytes, int64_t steps, Clock::time_point now) {
    size_t off = 0;
    if (bytes > alloc_.largest() || !alloc_.alloc(bytes, &off)) {
      stats_.rejected += 1;
      return KDE_E_BUDGET;
    }
    if (!stats_.have_first) {
      stats_.first = now;
      stats_.have_first = true;
    }
    sessions_.push_back(Session{ticket, off, bytes, steps, 0, false, false, now, now});
    return KDE_OK;
  }

  // Remove a queued request: KDE_OK (its outcome is KDE_E_CANCELLED),
  // KDE_E_AGAIN when it already runs, KDE_E_NOT_FOUND otherwise. An
  // attached session takes no further step: KDE_OK, and its ticket
  // completes with KDE_E_CANCELLED once the step in flight (if any) is
  // done, with the steps taken.
  kde_status cancel(uint64_t ticket, Clock::time_point now) {
    for (auto it = queue_.begin(); it != queue_.end(); ++it) {
      if (it->ticket != ticket) continue;
      Outcome o;
      o.status = KDE_E_CANCELLED;
      o.latency_s = o.queue_s = seconds(it->arrival, now);
      results_[ticket] = o;
      queue_.erase(it);
      work_.erase(ticket);
      ex_->forget(ticket);
      stats_.cancelled += 1;
      return KDE_OK;
    }
    for (const Slot& sl : slots_)
      for (const Request& r : sl.reqs)
        if (r.ticket == ticket) return KDE_E_AGAIN;
    for (Session& se : sessions_)
      if (se.ticket == ticket) {
        se.cancelled = true;
        return KDE_OK;
      }
    return KDE_E_NOT_FOUND;
  }

  // KDE_OK with the outcome once done, KDE_E_AGAIN while pending,
  // KDE_E_NOT_FOUND for a ticket never issued.
  kde_status poll(uint64_t ticket, Outcome* out) const {
    auto it = results_.find(ticket);
    if (it != results_.end()) {
      *out = it->second;
      return KDE_OK;
    }
    return known(ticket) ? KDE_E_AGAIN : KDE_E_NOT_FOUND;
  }

  // Progress: completed slots, session steps, admission. Returns true
  // while anything is queued, running or attached.
  bool tick(Clock::time_point now) {
    for (int k = 0; k < int(slots_.size()); ++k) {
      Slot& sl = slots_[size_t(k)];
      if (!sl.busy) continue;
      const kde_status q = ex_->poll(k);
      if (q == KDE_E_AGAIN) continue;
      std::vector<kde_status> st;
      if (q == KDE_OK) ex_->outcomes(k, &st);
      finish_slot(sl, q, st, now);
    }
    step_sessions(now);
    admit(now);
    return busy();
  }

  // Stop: queued requests are dropped (their outcome is KDE_E_CANCELLED),
  // nothing new starts, and attached sessions end after the step in flight.
  // tick() keeps finishing what runs until busy() turns false.
  void close(Clock::time_point now) {
    closing_ = true;
    while (!queue_.empty()) {
      const uint64_t t = queue_.front().ticket;
      (void)cancel(t, now);
    }
  }

  bool busy() const {
    if (!queue_.empty() || !sessions_.empty()) return true;
    for (const Slot& sl : slots_)
      if (sl.busy) return true;
    return false;
  }

  const Stats& stats() const { return stats_; }
  size_t queued() const { return queue_.size(); }
  size_t free_bytes() const { return alloc_.total_free(); }
  const std::vector<Slot>& slots() const { return slots_; }

 private:
  static bool joins(double cost, double head) { return cost <= 2.0 * head && cost >= 0.25 * head; }
  bool large(const Request& r) const { return r.cost >= cfg_.large_terms; }

  void complete(uint64_t ticket, const Outcome& o, Clock::time_point now) {
    results_[ticket] = o;
    if (o.status == KDE_OK) {
      stats_.completed += 1;
      stats_.latencies.push_back(o.latency_s);
      auto w = work_.find(ticket);
      if (w != work_.end()) {
        stats_.pair_evals += w->second.first;
        stats_.particles += w->second.second;
      }
    } else {
      stats_.failed += 1;
    }
    work_.erase(ticket);
    ex_->forget(ticket);
    stats_.last = now;
  }

  void finish_slot(Slot& sl, kde_status q, const std::vector<kde_status>& st, Clock::time_point now) {
    for (size_t k = 0; k < sl.reqs.size(); ++k) {
      const Request& r = sl.reqs[k];
      Outcome o;
      o.status = (q != KDE_OK) ? q : (k < st.size() ? st[k] : KDE_E_INTERNAL);
      o.batch_size = int32_t(sl.reqs.size());
      o.latency_s = seconds(r.arrival, now);
      o.queue_s = seconds(r.arrival, sl.started);
      o.run_s = seconds(sl.started, now);
      complete(r.ticket, o, now);
    }
    alloc_.release(sl.off, sl.bytes);
    sl.reqs.clear();
    sl.busy = false;
  }

  void step_sessions(Clock::time_point now) {
    for (size_t k = 0; k < sessions_.size();) {
      Session& se = sessions_[k];
      kde_status st = KDE_OK;
      bool finished = false;
      if (se.in_flight) {
        const kde_status q = ex_->session_poll(se.ticket);
        if (q == KDE_OK) {
          bool done = false;
          st = ex_->session_advance(se.ticket, &done);
          if (st == KDE_OK && done) {
            se.in_flight = false;
            se.steps_done += 1;
            se.steps_left -= 1;
            stats_.session_steps += 1;
            stats_.step_latencies.push_back(seconds(se.step_start, now));
          } else if (st != KDE_OK) {
            se.in_flight = false;
            se.steps_done += 1;  // a failed step is still a step taken
          }
        } else if (q != KDE_E_AGAIN) {
          st = q;
          se.in_flight = false;
        }
      }
      if (st == KDE_OK && !se.in_flight) {
        if (se.steps_left <= 0 || closing_ || se.cancelled) {
          finished = true;
          if (se.cancelled) st = KDE_E_CANCELLED;
        } else {
          se.step_start = now;
          st = ex_->session_begin(se.ticket);
          se.in_flight = (st == KDE_OK);
        }
      }
      if (st != KDE_OK || finished) {
        Outcome o;
        o.status = st;
        o.batch_size = 1;
        o.latency_s = o.run_s = seconds(se.arrival, now);
        o.steps = se.steps_done;
        results_[se.ticket] = o;
        if (st != KDE_OK && st != KDE_E_CANCELLED) stats_.failed += 1;
        alloc_.release(se.off, se.bytes);
        ex_->forget(se.ticket);
        stats_.last = now;
        sessions_.erase(sessions_.begin() + std::ptrdiff_t(k));
        continue;
      }
      ++k;
    }
  }

  void admit(Clock::time_point now) {
    if (closing_) return;
    for (int s = 0; s < int(slots_.size()); ++s) {
      Slot& sl = slots_[size_t(s)];
      if (queue_.empty()) return;
      if (sl.busy) continue;
      int large_running = 0;
      for (const Slot& o : slots_) large_running += (o.busy && o.large) ? 1 : 0;
      const bool large_ok = large_running < cfg_.large_slots;
      const size_t scan = std::min(queue_.size(), cfg_.scan);
      size_t h = scan;
      for (size_t k = 0; k < scan; ++k) {
        if (!large(queue_[k]) || large_ok) {
          h = k;
          break;
        }
      }
      if (h == scan) return;  // only large requests wait, and their slots are taken
      const bool head_large = large(queue_[h]);
      const double head = queue_[h].cost;
      const size_t room = alloc_.largest();
      std::vector<uint64_t> group;
      std::vector<size_t> taken;
      size_t group_bytes = 0;
      for (size_t k = h; k < scan && int(group.size()) < (head_large ? 1 : cfg_.max_batch); ++k) {
        if (k > h && (large(queue_[k]) || !joins(queue_[k].cost, head))) continue;
        group.push_back(queue_[k].ticket);
        size_t b = 0;
        if (!ex_->group_bytes(group, &b) || b > room) {
          group.pop_back();
          if (k == h) break;
          continue;
        }
        group_bytes = b;
        taken.push_back(k);
      }
      if (group.empty()) return;  // the head waits for arena space
      size_t off = 0;
      if (!alloc_.alloc(group_bytes, &off)) return;
      sl.busy = true;
      sl.large = head_large;
      sl.off = off;
      sl.bytes = group_bytes;
      sl.started = now;
      sl.reqs.clear();
      for (size_t k : taken) sl.reqs.push_back(queue_[k]);
      for (size_t k = taken.size(); k-- > 0;) queue_.erase(queue_.begin() + std::ptrdiff_t(taken[k]));
      stats_.launches += 1;
      stats_.batched += int64_t(group.size());
      const kde_status st = ex_->launch(s, group, off);
      if (st != KDE_OK) finish_slot(sl, st, {}, now);  // the group fails alone; the slot is free again
    }
  }

  Config cfg_;
  Executor* ex_;
  ArenaAlloc alloc_;
  std::vector<Slot> slots_;
  std::deque<Request> queue_;
  std::vector<Session> sessions_;
  std::unordered_map<uint64_t, Outcome> results_;
  std::unordered_map<uint64_t, std::pair<double, double>> work_;  // pair-evals and particles of a request
  uint64_t next_ticket_ = 1;
  bool closing_ = false;
  Stats stats_;
};

// p-quantile of a sample (linear interpolation between order statistics).
inline double quantile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p * double(v.size() - 1);
  const size_t i = size_t(pos);
  const double t = pos - double(i);
  return i + 1 < v.size() ? v[i] * (1.0 - t) + v[i + 1] * t : v[i];
}

}  // namespace sched
}  // namespace kde
