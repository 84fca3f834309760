// CPU driver of the server's host scheduling (csrc/sched.h) with a fake
// executor: a "solve" sleeps for its payload's duration.  No device code;
// prints one JSON object per scenario for tests/test_sched.py.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../paper_2110_08868_amd/csrc/sched.h"

using namespace mak::sched;

struct Fake {
  int ms = 0;
  int fail = 0;
};

// Holds a "workspace" like the server's slots: sized for the largest request
// it has run, given back when a much smaller one comes or when released.
// `resident` sums what every fake holds at this moment; `resident_peak` is its
// maximum, the fake's measured counterpart of the scheduler's bookkeeping.
struct FakeExec {
  static std::atomic<int> made, releases;
  static std::atomic<long long> resident, resident_peak;
  int slot;
  size_t holds = 0;
  explicit FakeExec(int s) : slot(s) { ++made; }
  ~FakeExec() { resident -= (long long)holds; }
  static size_t hold_after(size_t est, size_t held) {
    return (held > 0 && est * 2 < held) ? est : (est > held ? est : held);
  }
  void grow(size_t to) {
    resident += (long long)to - (long long)holds;
    holds = to;
    long long r = resident.load(), p = resident_peak.load();
    while (r > p && !resident_peak.compare_exchange_weak(p, r)) {
    }
  }
  void release() {
    ++releases;
    grow(0);
  }
  int run(Fake& f, std::string& err, int64_t est) {
    grow(hold_after(size_t(est), holds));
    std::this_thread::sleep_for(std::chrono::milliseconds(f.ms));
    if (f.fail) {
      err = "fake failure";
      return f.fail;
    }
    return 0;
  }
};
std::atomic<int> FakeExec::made{0};
std::atomic<int> FakeExec::releases{0};
std::atomic<long long> FakeExec::resident{0};
std::atomic<long long> FakeExec::resident_peak{0};

using Sched = RequestScheduler<Fake, FakeExec>;

static Sched::MakeExec maker() {
  return [](int32_t s) { return std::make_unique<FakeExec>(s); };
}

static void print_ticket(const Ticket<Fake>& t, double t0, bool last) {
  std::printf("{\"id\": %lld, \"est\": %zu, \"status\": %d, \"slot\": %d, \"submit\": %.6f, \"start\": %.6f, \"end\": %.6f}%s",
              (long long)t.id, t.est, t.status, t.slot, t.t_submit - t0, t.t_start - t0, t.t_end - t0,
              last ? "" : ", ");
}

static void print_stats(const Stats& s) {
  std::printf("\"stats\": {\"submitted\": %lld, \"completed\": %lld, \"queued\": %lld, \"active\": %d, "
              "\"peak_active\": %d, \"admitted_while_busy\": %lld, \"releases\": %lld, \"used\": %zu, "
              "\"peak_used\": %zu, \"budget\": %zu}",
              (long long)s.submitted, (long long)s.completed, (long long)s.queued, s.active, s.peak_active,
              (long long)s.admitted_while_busy, (long long)s.releases, s.used, s.peak_used, s.budget);
}

// Requests (est, ms) submitted at the given offsets (ms) into a scheduler.
static void scenario(size_t budget, int slots, const std::vector<std::vector<int>>& reqs) {
  const double t0 = now_s();
  Sched s(budget, slots, maker());
  std::vector<int64_t> ids;
  std::vector<std::string> errs;
  for (const auto& r : reqs) {
    const double due = t0 + r[2] * 1e-3;
    while (now_s() < due) std::this_thread::sleep_for(std::chrono::microseconds(200));
    Fake f;
    f.ms = r[1];
    f.fail = r.size() > 3 ? r[3] : 0;
    std::string err;
    ids.push_back(s.submit(f, size_t(r[0]), &err));
    errs.push_back(err);
  }
  std::vector<Ticket<Fake>> ts;
  for (int64_t id : ids) {
    Ticket<Fake> t;
    if (id >= 0 && s.wait(id, &t)) ts.push_back(t);
  }
  const Stats st = s.stats();
  s.shutdown();
  const Stats after = s.stats();
  std::printf("{\"ids\": [");
  for (size_t k = 0; k < ids.size(); ++k) std::printf("%lld%s", (long long)ids[k], k + 1 < ids.size() ? ", " : "");
  std::printf("], \"rejected_msg\": \"");
  for (const auto& e : errs)
    if (!e.empty()) std::printf("%s", e.c_str());
  std::printf("\", \"tickets\": [");
  for (size_t k = 0; k < ts.size(); ++k) print_ticket(ts[k], t0, k + 1 == ts.size());
  std::printf("], ");
  print_stats(st);
  std::printf(", \"executors\": %d, \"exec_releases\": %d, \"resident_peak\": %lld, "
              "\"used_after_shutdown\": %zu, \"resident_after_shutdown\": %lld}\n",
              FakeExec::made.load(), FakeExec::releases.load(), FakeExec::resident_peak.load(), after.used,
              FakeExec::resident.load());
}

// Threads post jobs to a Batcher whose run function takes `ms` per batch.
static void batcher_scenario(int threads, int posts, int ms) {
  Batcher<int> b;
  std::atomic<int> seen{0};
  std::vector<int> sizes;
  std::mutex mu;
  b.start([&](std::vector<int*>& jobs) {
    std::this_thread::sleep_for(std::chrono::milliseconds(ms));
    for (int* j : jobs) *j += 1;  // every job runs exactly once
    seen += int(jobs.size());
    std::lock_guard<std::mutex> lk(mu);
    sizes.push_back(int(jobs.size()));
  });
  std::vector<int> runs(size_t(threads * posts), 0);
  std::vector<std::thread> th;
  for (int t = 0; t < threads; ++t)
    th.emplace_back([&, t] {
      for (int k = 0; k < posts; ++k) b.post(&runs[size_t(t * posts + k)]);
    });
  for (auto& x : th) x.join();
  b.stop();
  int64_t nb = 0, nj = 0;
  int32_t mx = 0;
  b.counters(&nb, &nj, &mx);
  int once = 1;
  for (int r : runs) once = once && r == 1;
  std::printf("{\"batches\": %lld, \"jobs\": %lld, \"max_batch\": %d, \"every_job_once\": %d, \"seen\": %d}\n",
              (long long)nb, (long long)nj, mx, once, seen.load());
}

// Three threads post one job each, 20 ms apart, to a batcher that waits up
// to `window_ms` for as many jobs as there are threads.
static void window_scenario(int window_ms) {
  Batcher<int> b;
  b.start([&](std::vector<int*>& jobs) {
    for (int* j : jobs) *j += 1;
  });
  b.configure(int64_t(window_ms) * 1000, [] { return 3; });
  std::vector<int> runs(3, 0);
  std::vector<std::thread> th;
  for (int t = 0; t < 3; ++t)
    th.emplace_back([&, t] {
      std::this_thread::sleep_for(std::chrono::milliseconds(20 * t));
      b.post(&runs[size_t(t)]);
    });
  for (auto& x : th) x.join();
  b.stop();
  int64_t nb = 0, nj = 0;
  int32_t mx = 0;
  b.counters(&nb, &nj, &mx);
  std::printf("{\"batches\": %lld, \"jobs\": %lld, \"max_batch\": %d, \"every_job_once\": %d}\n",
              (long long)nb, (long long)nj, mx, int(runs[0] == 1 && runs[1] == 1 && runs[2] == 1));
}

int main(int argc, char** argv) {
  const std::string which = argc > 1 ? argv[1] : "";
  if (which == "budget") {
    // FIFO with memory admission: the 2nd (60) waits for the 1st (60); the
    // 3rd (30) stays behind the 2nd (no overtaking)
    scenario(100, 4, {{60, 80, 0}, {60, 40, 5}, {30, 10, 10}});
  } else if (which == "resident") {
    // workspaces stay charged after their requests end: the 60 after the
    // first pair reuses the idle 60 (no release); the 80 fits only once an
    // idle workspace is given back
    scenario(100, 2, {{60, 60, 0}, {30, 60, 5}, {60, 20, 150}, {80, 20, 250}});
  } else if (which == "overcommit") {
    // the pattern that overcommitted when only running requests counted: a
    // big request, then another big one while a small one holds the other
    // slot; idle workspaces keep being charged
    scenario(100, 3, {{70, 40, 0}, {20, 10, 5}, {70, 40, 10}, {20, 10, 15}, {70, 40, 20}});
  } else if (which == "reject") {
    scenario(100, 2, {{150, 10, 0}, {50, 10, 0}});
  } else if (which == "midflight") {
    // a long request, then short ones arriving while it runs
    scenario(0, 2, {{10, 300, 0}, {10, 20, 50}, {10, 20, 60}, {10, 20, 70}});
  } else if (which == "failure") {
    scenario(0, 2, {{10, 10, 0, 4}, {10, 10, 0}});
  } else if (which == "drain") {
    scenario(0, 3, {{1, 30, 0}, {1, 30, 0}, {1, 30, 0}, {1, 30, 0}, {1, 30, 0}, {1, 30, 0}, {1, 30, 0}});
  } else if (which == "batcher") {
    batcher_scenario(6, 20, 5);
  } else if (which == "window") {
    window_scenario(500);
  } else if (which == "nowindow") {
    window_scenario(0);
  } else {
    std::fprintf(stderr, "unknown scenario\n");
    return 2;
  }
  return 0;
}
