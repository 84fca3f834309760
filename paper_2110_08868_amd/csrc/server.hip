// Serving: many reconstruction requests of different sizes on one device.
//
// A FIFO queue feeds a fixed number of worker slots.  Each slot owns a
// library context (its device workspace stays resident and is reused by the
// next request) and its own HIP stream, and runs the Newton solve of one
// request at a time on that stream.  A request is admitted when a slot is
// free and its memory estimate fits in what the budget has left; requests
// arriving while others run are admitted as soon as slots and memory free
// up, and their kernels overlap on the device with the running ones.  Every
// solve is deterministic (fixed reduction orders, fixed clip order), so a
// request gives the same bits alone and in a mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mak.h"
#include "engine.h"

namespace {

// Packs the cell passes that solves post into shared launches.
struct PassBatcher final : mak::PassRunner {
  struct Posted {
    mak::PassJob job;
    bool done = false;
  };
  int device = 0;
  int precision = MAK_FP64;
  std::mutex mu;
  std::condition_variable cv_post, cv_done;
  std::deque<Posted*> posted;
  bool stopping = false;
  int64_t batches = 0, passes = 0;
  int32_t max_batch = 0;
  std::thread th;

  void start(int dev, int prec) {
    device = dev;
    precision = prec;
    th = std::thread([this] { loop(); });
  }
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stopping = true;
    }
    cv_post.notify_all();
    if (th.joinable()) th.join();
  }
  void loop() {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    std::vector<Posted*> take;
    std::vector<mak::PassJob*> jobs;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_post.wait(lk, [&] { return stopping || !posted.empty(); });
        if (posted.empty()) break;  // stopping with nothing posted
        take.assign(posted.begin(), posted.end());
        posted.clear();
      }
      jobs.clear();
      for (Posted* p : take) jobs.push_back(&p->job);
      try {
        mak::run_cells_batch(jobs.data(), int(jobs.size()), precision, st);
      } catch (const mak::Error& e) {  // a device error: every job of the batch fails
        for (mak::PassJob* j : jobs) {
          j->status = e.status;
          j->err = e.msg;
        }
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        for (Posted* p : take) p->done = true;
        ++batches;
        passes += int64_t(take.size());
        if (int32_t(take.size()) > max_batch) max_batch = int32_t(take.size());
      }
      cv_done.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
  }
  // Called by a solve on its worker thread.
  mak::ClipStats run(mak::PointSet& ps, mak::CellPass& out, int prec, bool faces, hipStream_t st,
                     bool tolerate) override {
    if (prec != precision) MAK_FAIL(MAK_EINVAL, "pass precision differs from the server's");
    // the solve's own stream wrote the weights: they must be on the device
    MAK_HIP(hipStreamSynchronize(st));
    Posted p;
    p.job.ps = &ps;
    p.job.out = &out;
    p.job.faces = faces;
    p.job.tolerate = tolerate;
    {
      std::unique_lock<std::mutex> lk(mu);
      posted.push_back(&p);
      cv_post.notify_all();
      cv_done.wait(lk, [&] { return p.done; });
    }
    if (p.job.status != MAK_OK) MAK_FAIL(p.job.status, p.job.err);
    return p.job.cs;
  }
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  const double* points = nullptr;
  int64_t N = 0;
  double L = 0, tol = 0;
  double* psi = nullptr;
  double* cent = nullptr;
  double* disp = nullptr;
  size_t est = 0;
  bool done = false;
  mak_status status = MAK_OK;
  mak_solve_info info{};
  std::string err;
  double t_submit = 0, t_start = 0, t_end = 0;
  int32_t slot = -1;
};

}  // namespace

struct mak_server {
  int device = 0;
  mak_options opt{};
  size_t budget = 0;
  int32_t slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<int64_t, std::shared_ptr<Request>> reqs;
  size_t used = 0, peak_used = 0;
  int32_t active = 0, peak_active = 0;
  int64_t next_id = 1, submitted = 0, completed = 0, overlapped = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::string err;
  PassBatcher batcher;

  void worker(int32_t slot) {
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    mak_ctx* ctx = nullptr;
    size_t ctx_est = 0;  // estimate of the largest request the context has served
    for (;;) {
      std::shared_ptr<Request> r;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          return (!queue.empty() && used + queue.front()->est <= budget) ||
                 (stopping && queue.empty());
        });
        if (queue.empty()) break;  // stopping with nothing left
        r = queue.front();
        queue.pop_front();
        used += r->est;
        if (used > peak_used) peak_used = used;
        if (active > 0) ++overlapped;
        ++active;
        if (active > peak_active) peak_active = active;
        r->t_start = now_s();
        r->slot = slot;
        // admit the next one too if it fits (another worker)
        cv_work.notify_all();
      }
      // a much smaller request releases the workspace sized for a larger one
      if (ctx && r->est * 2 < ctx_est) {
        mak_destroy(ctx);
        ctx = nullptr;
      }
      if (!ctx) {
        if (mak_create(&ctx, device, &opt) != MAK_OK) ctx = nullptr;
        if (ctx) mak::set_pass_runner(ctx, &batcher);
        ctx_est = 0;
      }
      if (r->est > ctx_est) ctx_est = r->est;
      mak_status s = MAK_EHIP;
      std::string msg = "context creation failed";
      mak_solve_info info{};
      if (ctx) {
        s = mak_solve(ctx, r->points, r->N, r->L, r->tol, r->psi, r->cent, r->disp, &info, st);
        msg = s == MAK_OK ? "" : mak_last_error(ctx);
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        r->status = s;
        r->err = msg;
        r->info = info;
        r->t_end = now_s();
        r->done = true;
        used -= r->est;
        --active;
        ++completed;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (ctx) mak_destroy(ctx);
    if (st) (void)hipStreamDestroy(st);
  }
};

extern "C" {

mak_status mak_server_create(mak_server** out, int device, const mak_options* opt,
                             size_t mem_budget_bytes, int32_t max_slots) {
  if (!out || max_slots < 1 || max_slots > 64) return MAK_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return MAK_EHIP;
  }
  mak_server* s = new mak_server();
  s->device = device;
  mak_default_options(&s->opt);
  if (opt) s->opt = *opt;
  s->budget = mem_budget_bytes ? mem_budget_bytes : ~size_t(0);
  s->slots = max_slots;
  s->batcher.start(device, s->opt.precision);
  for (int32_t k = 0; k < max_slots; ++k) s->workers.emplace_back([s, k] { s->worker(k); });
  *out = s;
  return MAK_OK;
}

mak_status mak_server_submit(mak_server* s, const double* points, int64_t N, double L, double tol,
                             double* psi, double* centroids, double* displacements, int64_t* req_id) {
  if (!s || !points || !psi || !centroids || !displacements || !req_id || N < 1 || !(L > 0) ||
      !(tol > 0))
    return MAK_EINVAL;
  auto r = std::make_shared<Request>();
  r->points = points;
  r->N = N;
  r->L = L;
  r->tol = tol;
  r->psi = psi;
  r->cent = centroids;
  r->disp = displacements;
  r->est = mak_solve_memory_estimate(N, s->opt.precision);
  std::lock_guard<std::mutex> lk(s->mu);
  if (r->est > s->budget) {
    s->err = "request needs " + std::to_string(r->est) + " bytes, budget is " + std::to_string(s->budget);
    return MAK_ENOMEM;
  }
  r->id = s->next_id++;
  r->t_submit = now_s();
  s->reqs[r->id] = r;
  s->queue.push_back(r);
  ++s->submitted;
  *req_id = r->id;
  s->cv_work.notify_all();
  return MAK_OK;
}

mak_status mak_server_poll(mak_server* s, int64_t req_id, int32_t* done, mak_solve_info* info,
                           double* times) {
  if (!s || !done) return MAK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return MAK_ENOTFOUND;
  const Request& r = *it->second;
  *done = r.done ? 1 : 0;
  if (times) {
    times[0] = r.t_submit;
    times[1] = r.t_start;
    times[2] = r.t_end;
  }
  if (!r.done) return MAK_OK;
  if (info) *info = r.info;
  return r.status;
}

mak_status mak_server_wait(mak_server* s, int64_t req_id, mak_solve_info* info, double* times) {
  if (!s) return MAK_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return MAK_ENOTFOUND;
  std::shared_ptr<Request> r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  if (info) *info = r->info;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_start;
    times[2] = r->t_end;
  }
  if (r->status != MAK_OK) s->err = r->err;
  return r->status;
}

mak_status mak_server_release(mak_server* s, int64_t req_id) {
  if (!s) return MAK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return MAK_ENOTFOUND;
  if (!it->second->done) return MAK_EINVAL;
  s->reqs.erase(it);
  return MAK_OK;
}

mak_status mak_server_stats(mak_server* s, mak_server_info* out) {
  if (!s || !out) return MAK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->queued = int64_t(s->queue.size());
  out->active = s->active;
  out->peak_active = s->peak_active;
  out->admitted_while_busy = s->overlapped;
  out->used_bytes = s->used;
  out->peak_used_bytes = s->peak_used;
  out->budget_bytes = s->budget;
  {
    std::lock_guard<std::mutex> lb(s->batcher.mu);
    out->pass_batches = s->batcher.batches;
    out->batched_passes = s->batcher.passes;
    out->max_batch = s->batcher.max_batch;
  }
  return MAK_OK;
}

const char* mak_server_last_error(const mak_server* s) { return s ? s->err.c_str() : ""; }

void mak_server_destroy(mak_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  s->batcher.stop();
  delete s;
}

}  // extern "C"
