// Host-side scheduling of the server, free of device code so that it can be
// exercised on the CPU with a fake executor.
//
// RequestScheduler: a FIFO queue feeding `slots` worker threads.  Each
// worker owns one executor for its whole life, and an executor keeps its
// device workspace between requests, so the budget is charged with what the
// executors hold, not only with what is running: a slot's holding is charged
// from the request that sizes it until the executor releases it.  The head
// request is admitted on a free worker when the total held after it (that
// worker's holding replaced by what it will hold once sized for the request)
// fits in the budget; an idle worker whose holding keeps the head request
// out releases its workspace.  No overtaking: a large head request is not
// starved by smaller ones behind it.  A request submitted while others run
// starts as soon as a worker and memory free up.
//
// Batcher: solves post jobs (cell passes) and block; one thread takes every
// job posted so far at once (optionally after a short window in which more
// may arrive) and hands them to the run function together.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace mak {
namespace sched {

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Stats {
  int64_t submitted = 0, completed = 0, queued = 0;
  int32_t active = 0, peak_active = 0;
  int64_t admitted_while_busy = 0;
  int64_t releases = 0;  // idle workspaces released to admit the head request
  size_t used = 0, peak_used = 0, budget = 0;  // bytes held by the executors
};

template <class P>
struct Ticket {
  int64_t id = 0;
  size_t est = 0;
  P payload{};
  bool done = false;
  int status = 0;  // 0 = success, else the executor's error code
  std::string err;
  double t_submit = 0, t_start = 0, t_end = 0;
  int32_t slot = -1;
};

// Exec: constructed once per worker.
//   int run(P&, std::string& err, int64_t est)  runs one request, returns 0 or
//                                               an error code;
//   static size_t hold_after(size_t est, size_t held)
//                                               bytes an executor holding
//                                               `held` holds once it has run
//                                               a request of estimate est;
//   void release()                              frees what it holds (idle).
template <class P, class Exec>
class RequestScheduler {
 public:
  using MakeExec = std::function<std::unique_ptr<Exec>(int32_t slot)>;

  RequestScheduler(size_t budget, int32_t slots, MakeExec make)
      : make_(std::move(make)), held_(size_t(slots), 0), idle_(size_t(slots), false) {
    budget_ = budget ? budget : ~size_t(0);
    for (int32_t k = 0; k < slots; ++k) workers_.emplace_back([this, k] { worker(k); });
  }
  ~RequestScheduler() { shutdown(); }
  RequestScheduler(const RequestScheduler&) = delete;
  RequestScheduler& operator=(const RequestScheduler&) = delete;

  // Queue a request; returns its id, or -1 when the estimate exceeds the
  // whole budget (it could never run).
  int64_t submit(P payload, size_t est, std::string* err) {
    std::lock_guard<std::mutex> lk(mu_);
    if (est > budget_) {
      if (err) *err = "request needs " + std::to_string(est) + " bytes, budget is " + std::to_string(budget_);
      return -1;
    }
    auto t = std::make_shared<Ticket<P>>();
    t->id = next_id_++;
    t->est = est;
    t->payload = std::move(payload);
    t->t_submit = now_s();
    tickets_[t->id] = t;
    queue_.push_back(t);
    ++submitted_;
    cv_work_.notify_all();
    return t->id;
  }
  // false: unknown id.  *out is a copy of the ticket.
  bool poll(int64_t id, Ticket<P>* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return false;
    if (out) *out = *it->second;
    return true;
  }
  bool wait(int64_t id, Ticket<P>* out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return false;
    std::shared_ptr<Ticket<P>> t = it->second;
    cv_done_.wait(lk, [&] { return t->done; });
    if (out) *out = *t;
    return true;
  }
  // Forget a finished request: 0 ok, 1 unknown, 2 still running.
  int release(int64_t id) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(id);
    if (it == tickets_.end()) return 1;
    if (!it->second->done) return 2;
    tickets_.erase(it);
    return 0;
  }
  Stats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    Stats s;
    s.submitted = submitted_;
    s.completed = completed_;
    s.queued = int64_t(queue_.size());
    s.active = active_;
    s.peak_active = peak_active_;
    s.admitted_while_busy = overlapped_;
    s.releases = releases_;
    s.used = used_;
    s.peak_used = peak_used_;
    s.budget = budget_;
    return s;
  }
  // Finish everything queued and running, then join the workers.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) return;
      stopping_ = true;
    }
    cv_work_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  // Whether the idle worker `k` can take the head request without releasing
  // anything, and what it would hold then.
  bool fits(int32_t k, size_t* after) const {
    const size_t a = Exec::hold_after(queue_.front()->est, held_[size_t(k)]);
    if (after) *after = a;
    return used_ - held_[size_t(k)] + a <= budget_;
  }
  bool some_idle_fits() const {
    for (size_t k = 0; k < idle_.size(); ++k)
      if (idle_[k] && fits(int32_t(k), nullptr)) return true;
    return false;
  }

  void worker(int32_t slot) {
    std::unique_ptr<Exec> ex = make_(slot);
    const size_t k = size_t(slot);
    for (;;) {
      std::shared_ptr<Ticket<P>> t;
      {
        std::unique_lock<std::mutex> lk(mu_);
        idle_[k] = true;
        size_t after = 0;
        for (;;) {
          if (queue_.empty()) {
            if (stopping_) break;
            cv_work_.wait(lk);
            continue;
          }
          if (fits(slot, &after)) break;
          if (held_[k] > 0 && ex && !some_idle_fits()) {
            // no idle worker can take the head request as things are, and
            // what this one holds keeps it out: give the workspace back
            const size_t h = held_[k];
            idle_[k] = false;  // not a candidate while it releases
            lk.unlock();
            ex->release();
            lk.lock();
            idle_[k] = true;
            used_ -= h;
            held_[k] = 0;
            ++releases_;
            cv_work_.notify_all();
            continue;
          }
          cv_work_.wait(lk);
        }
        if (queue_.empty()) {  // stopping with nothing left
          idle_[k] = false;
          break;
        }
        t = queue_.front();
        queue_.pop_front();
        idle_[k] = false;
        used_ = used_ - held_[k] + after;
        held_[k] = after;
        if (used_ > peak_used_) peak_used_ = used_;
        if (active_ > 0) ++overlapped_;
        ++active_;
        if (active_ > peak_active_) peak_active_ = active_;
        t->t_start = now_s();
        t->slot = slot;
        cv_work_.notify_all();  // the next one may fit too (another worker)
      }
      std::string err;
      const int status = ex ? ex->run(t->payload, err, int64_t(t->est)) : -1;
      {
        std::lock_guard<std::mutex> lk(mu_);
        t->status = status;
        t->err = ex ? err : "executor could not be created";
        t->t_end = now_s();
        t->done = true;
        --active_;
        ++completed_;
      }
      cv_done_.notify_all();
      cv_work_.notify_all();
    }
    ex.reset();  // the executor's workspace goes with it
    std::lock_guard<std::mutex> lk(mu_);
    used_ -= held_[k];
    held_[k] = 0;
  }

  MakeExec make_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<std::shared_ptr<Ticket<P>>> queue_;
  std::map<int64_t, std::shared_ptr<Ticket<P>>> tickets_;
  std::vector<size_t> held_;  // per worker: bytes its executor holds (in used_)
  std::vector<bool> idle_;    // per worker: waiting for a request
  size_t budget_ = 0, used_ = 0, peak_used_ = 0;
  int32_t active_ = 0, peak_active_ = 0;
  int64_t next_id_ = 1, submitted_ = 0, completed_ = 0, overlapped_ = 0, releases_ = 0;
  bool stopping_ = false;
  std::vector<std::thread> workers_;
};

template <class Job>
class Batcher {
 public:
  using RunFn = std::function<void(std::vector<Job*>&)>;

  // init / fini run on the batcher thread (device and stream set-up).
  void start(RunFn run, std::function<void()> init = {}, std::function<void()> fini = {}) {
    run_ = std::move(run);
    th_ = std::thread([this, init, fini] {
      if (init) init();
      loop();
      if (fini) fini();
    });
  }
  // After the first posted job the batcher may wait up to `window_us` for
  // more, until `expect()` jobs are posted (e.g. the number of solves in
  // flight: when all of them wait for a pass, nothing else will come).
  // 0 (the default): run what is posted at once.
  void configure(int64_t window_us, std::function<int()> expect) {
    std::lock_guard<std::mutex> lk(mu_);
    window_us_ = window_us;
    expect_ = std::move(expect);
  }
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_post_.notify_all();
    if (th_.joinable()) th_.join();
  }
  // Blocks until the batch that took `j` has run.
  void post(Job* j) {
    Posted p{j, false};
    std::unique_lock<std::mutex> lk(mu_);
    posted_.push_back(&p);
    cv_post_.notify_all();
    cv_done_.wait(lk, [&] { return p.done; });
  }
  void counters(int64_t* batches, int64_t* jobs, int32_t* max_batch) {
    std::lock_guard<std::mutex> lk(mu_);
    *batches = batches_;
    *jobs = jobs_;
    *max_batch = max_batch_;
  }

 private:
  struct Posted {
    Job* job;
    bool done;
  };
  void loop() {
    std::vector<Posted*> take;
    std::vector<Job*> jobs;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_post_.wait(lk, [&] { return stopping_ || !posted_.empty(); });
        if (posted_.empty()) break;  // stopping with nothing posted
        if (window_us_ > 0) {
          const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(window_us_);
          cv_post_.wait_until(lk, until, [&] {
            return stopping_ || int(posted_.size()) >= (expect_ ? expect_() : 1);
          });
        }
        take.assign(posted_.begin(), posted_.end());
        posted_.clear();
      }
      jobs.clear();
      for (Posted* p : take) jobs.push_back(p->job);
      run_(jobs);
      {
        std::lock_guard<std::mutex> lk(mu_);
        for (Posted* p : take) p->done = true;
        ++batches_;
        jobs_ += int64_t(take.size());
        if (int32_t(take.size()) > max_batch_) max_batch_ = int32_t(take.size());
      }
      cv_done_.notify_all();
    }
  }

  RunFn run_;
  std::mutex mu_;
  std::condition_variable cv_post_, cv_done_;
  std::deque<Posted*> posted_;
  bool stopping_ = false;
  int64_t window_us_ = 0;
  std::function<int()> expect_;
  int64_t batches_ = 0, jobs_ = 0;
  int32_t max_batch_ = 0;
  std::thread th_;
};

}  // namespace sched
}  // namespace mak
