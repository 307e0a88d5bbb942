// Host test of the request server's scheduler (paper_1804_11174_amd/csrc/
// sched.hpp) against a fake device: admission and batching, the budget,
// cancellation, failure isolation, per-request numeric status, attached
// sessions, closing, and a threaded run (submitters, pollers and a ticking
// worker sharing one mutex, as the server does) for the thread sanitizer.
// Exits non-zero with a message on the first failed check.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sched.hpp"

using namespace kde;
using namespace kde::sched;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// A fake device: a group completes after `latency` polls of its slot; a
// session step after `step_polls` polls (every third step asks for a
// second wait, as a step whose rule fires does).
struct FakeDevice : Executor {
  std::unordered_map<uint64_t, size_t> bytes;  // per request
  std::set<uint64_t> bad_launch, bad_poll, nan;
  std::unordered_map<int, std::vector<uint64_t>> running;
  std::unordered_map<int, int> polls_left;
  std::unordered_map<uint64_t, int> sess_polls, sess_steps;
  std::set<uint64_t> sess_fail_at_step, scanning;
  std::vector<std::vector<uint64_t>> launched;
  int latency = 3, step_polls = 2;
  int forgotten = 0;

  bool group_bytes(const std::vector<uint64_t>& t, size_t* b) override {
    size_t s = 0;
    for (uint64_t k : t) s += bytes.at(k);
    *b = s;
    return true;
  }
  kde_status launch(int slot, const std::vector<uint64_t>& t, size_t) override {
    for (uint64_t k : t)
      if (bad_launch.count(k)) return KDE_E_HIP;
    running[slot] = t;
    polls_left[slot] = latency;
    launched.push_back(t);
    return KDE_OK;
  }
  kde_status poll(int slot) override {
    if (--polls_left[slot] > 0) return KDE_E_AGAIN;
    for (uint64_t k : running[slot])
      if (bad_poll.count(k)) return KDE_E_HIP;
    return KDE_OK;
  }
  void outcomes(int slot, std::vector<kde_status>* st) override {
    st->clear();
    for (uint64_t k : running[slot]) st->push_back(nan.count(k) ? KDE_E_NUMERIC : KDE_OK);
  }
  void forget(uint64_t) override { ++forgotten; }
  kde_status session_begin(uint64_t t) override {
    sess_polls[t] = step_polls;
    return KDE_OK;
  }
  kde_status session_poll(uint64_t t) override { return --sess_polls[t] > 0 ? KDE_E_AGAIN : KDE_OK; }
  kde_status session_advance(uint64_t t, bool* done) override {
    const int k = ++sess_steps[t];
    if (sess_fail_at_step.count(t) && k == 2) {
      *done = true;
      return KDE_E_NUMERIC;
    }
    if (k % 3 == 0 && !scanning.count(t)) {  // the rule fired: one more wait
      scanning.insert(t);
      sess_polls[t] = step_polls;
      sess_steps[t] -= 1;
      *done = false;
      return KDE_OK;
    }
    scanning.erase(t);
    *done = true;
    return KDE_OK;
  }
};

static Config cfg(size_t budget, int nslots = 2, int max_batch = 4) {
  Config c;
  c.nslots = nslots;
  c.max_batch = max_batch;
  c.large_slots = 1;
  c.large_terms = 1e9;
  c.budget = budget;
  return c;
}

static uint64_t add(Scheduler& s, FakeDevice& d, double cost, size_t bytes, Clock::time_point now) {
  const uint64_t t = s.new_ticket();
  d.bytes[t] = bytes;
  CHECK(s.submit(t, cost, bytes, now, 1.0, 1.0) == KDE_OK);
  return t;
}

static void run(Scheduler& s, Clock::time_point& now, int max_ticks = 10000) {
  for (int k = 0; k < max_ticks && s.tick(now); ++k) now += std::chrono::microseconds(10);
  CHECK(!s.busy());
}

static void test_batching_and_large_order() {
  FakeDevice d;
  Scheduler s(cfg(1 << 20), &d);
  auto now = Clock::now();
  std::vector<uint64_t> small;
  for (int k = 0; k < 6; ++k) small.push_back(add(s, d, 1e6 * (1 + 0.1 * k), 1000, now));
  const uint64_t big1 = add(s, d, 5e9, 1000, now), big2 = add(s, d, 6e9, 1000, now);
  run(s, now);
  // the small ones went in groups of at most max_batch; the large ones alone, in order
  size_t in_groups = 0;
  int pos1 = -1, pos2 = -1;
  for (size_t g = 0; g < d.launched.size(); ++g) {
    CHECK(d.launched[g].size() <= 4);
    for (uint64_t t : d.launched[g]) {
      if (t == big1) { CHECK(d.launched[g].size() == 1); pos1 = int(g); }
      if (t == big2) { CHECK(d.launched[g].size() == 1); pos2 = int(g); }
    }
    if (d.launched[g].size() > 1) in_groups += d.launched[g].size();
  }
  CHECK(in_groups >= 4);  // small requests of similar cost were admitted together
  CHECK(pos1 >= 0 && pos2 > pos1);
  for (uint64_t t : small) {
    Outcome o;
    CHECK(s.poll(t, &o) == KDE_OK && o.status == KDE_OK && o.batch_size >= 1);
  }
  CHECK(s.stats().completed == 8 && s.stats().failed == 0);
  CHECK(s.free_bytes() == (1u << 20));
}

static void test_budget() {
  FakeDevice d;
  Scheduler s(cfg(4096, 4, 8), &d);
  auto now = Clock::now();
  const uint64_t t = s.new_ticket();
  CHECK(s.submit(t, 1e6, 5000, now, 1, 1) == KDE_E_BUDGET);
  CHECK(s.stats().rejected == 1);
  // two requests of 3000 bytes cannot run together: the second waits
  const uint64_t a = add(s, d, 1e6, 3000, now), b = add(s, d, 1e6, 3000, now);
  s.tick(now);
  CHECK(d.launched.size() == 1 && d.launched[0].size() == 1 && d.launched[0][0] == a);
  run(s, now);
  CHECK(d.launched.size() == 2 && d.launched[1][0] == b);
}

static void test_cancel() {
  FakeDevice d;
  Scheduler s(cfg(4096, 1, 1), &d);
  auto now = Clock::now();
  const uint64_t a = add(s, d, 1e6, 1000, now), b = add(s, d, 1e6, 1000, now);
  s.tick(now);  // a runs, b waits
  CHECK(s.cancel(a, now) == KDE_E_AGAIN);
  CHECK(s.cancel(b, now) == KDE_OK);
  CHECK(s.cancel(b, now) == KDE_E_NOT_FOUND);
  CHECK(s.cancel(12345, now) == KDE_E_NOT_FOUND);
  run(s, now);
  Outcome o;
  CHECK(s.poll(b, &o) == KDE_OK && o.status == KDE_E_CANCELLED);
  CHECK(s.poll(a, &o) == KDE_OK && o.status == KDE_OK);
  CHECK(s.poll(777, &o) == KDE_E_NOT_FOUND);
  CHECK(s.stats().cancelled == 1 && s.stats().completed == 1);
  CHECK(d.launched.size() == 1);
}

static void test_failure_isolation_and_numeric() {
  FakeDevice d;
  Scheduler s(cfg(1 << 20, 2, 1), &d);
  auto now = Clock::now();
  const uint64_t a = add(s, d, 1e6, 100, now), b = add(s, d, 1e6, 100, now), c = add(s, d, 1e6, 100, now),
                 e = add(s, d, 1e6, 100, now);
  d.bad_launch.insert(a);
  d.bad_poll.insert(b);
  d.nan.insert(c);
  run(s, now);
  Outcome o;
  CHECK(s.poll(a, &o) == KDE_OK && o.status == KDE_E_HIP);
  CHECK(s.poll(b, &o) == KDE_OK && o.status == KDE_E_HIP);
  CHECK(s.poll(c, &o) == KDE_OK && o.status == KDE_E_NUMERIC);
  CHECK(s.poll(e, &o) == KDE_OK && o.status == KDE_OK);
  // only the request that succeeded counts as completed and enters the latencies
  CHECK(s.stats().completed == 1 && s.stats().failed == 3 && s.stats().latencies.size() == 1);
  CHECK(s.free_bytes() == (1u << 20));
}

static void test_sessions() {
  FakeDevice d;
  Scheduler s(cfg(10000, 2, 4), &d);
  auto now = Clock::now();
  const uint64_t s1 = s.new_ticket();
  CHECK(s.attach(s1, 6000, 7, now) == KDE_OK);
  CHECK(s.free_bytes() == 10000 - 6144);
  const uint64_t s2 = s.new_ticket();
  CHECK(s.attach(s2, 6000, 3, now) == KDE_E_BUDGET);
  const uint64_t s3 = s.new_ticket();
  d.sess_fail_at_step.insert(s3);
  CHECK(s.attach(s3, 1000, 5, now) == KDE_OK);
  const uint64_t r = add(s, d, 1e6, 5000, now);  // does not fit while s1 is attached
  run(s, now);
  Outcome o;
  CHECK(s.poll(s1, &o) == KDE_OK && o.status == KDE_OK && o.steps == 7);
  CHECK(s.poll(s3, &o) == KDE_OK && o.status == KDE_E_NUMERIC && o.steps == 2);
  CHECK(s.poll(r, &o) == KDE_OK && o.status == KDE_OK);
  CHECK(s.stats().session_steps == 7 + 1 && s.stats().step_latencies.size() == 8);
  CHECK(s.free_bytes() == 10000);
}

// Cancelling an attached session detaches it after the step in flight.
static void test_session_detach() {
  FakeDevice d;
  Scheduler s(cfg(10000, 1, 1), &d);
  auto now = Clock::now();
  const uint64_t se = s.new_ticket();
  CHECK(s.attach(se, 4000, 1000000, now) == KDE_OK);
  for (int k = 0; k < 20; ++k) {
    s.tick(now);
    now += std::chrono::microseconds(10);
  }
  CHECK(s.cancel(se, now) == KDE_OK);
  CHECK(s.cancel(se, now) == KDE_OK);  // still attached until its step ends
  run(s, now);
  Outcome o;
  CHECK(s.poll(se, &o) == KDE_OK && o.status == KDE_E_CANCELLED);
  CHECK(o.steps >= 1 && o.steps < 1000000 && o.steps == s.stats().session_steps);
  CHECK(s.cancel(se, now) == KDE_E_NOT_FOUND);
  CHECK(s.free_bytes() == 10000 && s.stats().failed == 0 && s.stats().cancelled == 0);
}

static void test_close() {
  FakeDevice d;
  Scheduler s(cfg(1 << 20, 1, 1), &d);
  auto now = Clock::now();
  const uint64_t a = add(s, d, 1e6, 100, now), b = add(s, d, 1e6, 100, now);
  const uint64_t se = s.new_ticket();
  CHECK(s.attach(se, 100, 1000, now) == KDE_OK);
  s.tick(now);
  s.close(now);
  run(s, now);
  Outcome o;
  CHECK(s.poll(a, &o) == KDE_OK && o.status == KDE_OK);
  CHECK(s.poll(b, &o) == KDE_OK && o.status == KDE_E_CANCELLED);
  CHECK(s.poll(se, &o) == KDE_OK && o.status == KDE_OK && o.steps < 1000);
}

// Submitters and pollers on their own threads, a worker ticking, all under
// one mutex (the server's locking).
static void test_threads() {
  FakeDevice d;
  d.latency = 2;
  Scheduler s(cfg(1 << 16, 4, 8), &d);
  std::mutex mu;
  std::atomic<bool> stop{false};
  std::thread worker([&] {
    while (!stop.load()) {
      std::lock_guard<std::mutex> lk(mu);
      s.tick(Clock::now());
    }
  });
  const int kThreads = 4, kPer = 200;
  std::vector<std::vector<uint64_t>> tickets(kThreads);
  std::vector<std::thread> th;
  for (int k = 0; k < kThreads; ++k)
    th.emplace_back([&, k] {
      for (int r = 0; r < kPer; ++r) {
        std::lock_guard<std::mutex> lk(mu);
        const uint64_t t = s.new_ticket();
        d.bytes[t] = 256 + 64 * (r % 7);
        CHECK(s.submit(t, 1e6 * (1 + (r % 3)), d.bytes[t], Clock::now(), 1, 1) == KDE_OK);
        tickets[size_t(k)].push_back(t);
        if (r % 50 == 7) (void)s.cancel(t, Clock::now());
      }
    });
  for (auto& t : th) t.join();
  for (int k = 0; k < kThreads; ++k)
    for (uint64_t t : tickets[size_t(k)]) {
      for (;;) {
        std::lock_guard<std::mutex> lk(mu);
        Outcome o;
        const kde_status st = s.poll(t, &o);
        if (st == KDE_OK) {
          CHECK(o.status == KDE_OK || o.status == KDE_E_CANCELLED);
          break;
        }
        CHECK(st == KDE_E_AGAIN);
      }
    }
  stop.store(true);
  worker.join();
  std::lock_guard<std::mutex> lk(mu);
  CHECK(s.stats().completed + s.stats().cancelled == kThreads * kPer);
  CHECK(!s.busy() && s.free_bytes() == (1u << 16));
}

int main() {
  test_batching_and_large_order();
  test_budget();
  test_cancel();
  test_failure_isolation_and_numeric();
  test_sessions();
  test_session_detach();
  test_close();
  test_threads();
  std::printf("sched tests ok\n");
  return 0;
}
