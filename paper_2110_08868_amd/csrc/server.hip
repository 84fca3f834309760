// Serving: many reconstruction requests of different sizes on one device.
//
// Admission and workers come from sched.h: a FIFO queue feeds a fixed number
// of worker slots.  Each slot owns a library context (its device workspace
// stays resident and is reused by the next request) and its own HIP stream,
// on which the Newton and PCG work of its request runs.  The budget is
// charged with the workspaces the slots hold, idle or not; the head request
// starts when a slot is free and the holdings with that slot's workspace
// resized for it fit in the budget (idle slots give their workspace back
// when no idle slot can take it), so requests arriving while others run are
// admitted as soon as slots and memory free up.
//
// Cell passes go through the pass batcher: a solve that needs one posts it
// and waits; the batcher thread takes every posted pass at once (with a
// batch window, after waiting up to that long until every solve in flight
// has posted) and runs them in shared clip launches on its own stream (each
// stage launch carries up to kMaxJobs point sets), so concurrent requests
// share launches.  Every solve
// is deterministic (fixed reduction orders, fixed clip order, a cell's result
// independent of the other cells in its launch), so a request gives the same
// bits alone and in a mix.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>

#include "../../include/mak.h"
#include "engine.h"
#include "sched.h"

namespace {

struct SolveArgs {
  const double* points = nullptr;
  int64_t N = 0;
  double L = 0, tol = 0;
  double* psi = nullptr;
  double* cent = nullptr;
  double* disp = nullptr;
  mak_solve_info info{};
};

// The cell-pass side of the server: a sched::Batcher of PassJobs run by
// run_cells_batch on the batcher's stream.
struct PassBatcher final : mak::PassRunner {
  int device = 0;
  int precision = MAK_FP64;
  hipStream_t st = nullptr;
  mak::sched::Batcher<mak::PassJob> b;

  void start(int dev, int prec) {
    device = dev;
    precision = prec;
    b.start(
        [this](std::vector<mak::PassJob*>& jobs) {
          try {
            mak::run_cells_batch(jobs.data(), int(jobs.size()), precision, st);
          } catch (const mak::Error& e) {  // a device error: every job of the batch fails
            for (mak::PassJob* j : jobs) {
              j->status = e.status;
              j->err = e.msg;
            }
          }
        },
        [this] {
          (void)hipSetDevice(device);
          (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        },
        [this] {
          if (st) (void)hipStreamDestroy(st);
        });
  }
  // Called by a solve on its worker thread.
  mak::ClipStats run(mak::PointSet& ps, mak::CellPass& out, const mak::PassOpts& o,
                     hipStream_t sst) override {
    if (o.precision != precision) MAK_FAIL(MAK_EINVAL, "pass precision differs from the server's");
    // the solve's own stream wrote the weights: they must be on the device
    MAK_HIP(hipStreamSynchronize(sst));
    mak::PassJob job;
    job.ps = &ps;
    job.out = &out;
    job.opt = o;
    b.post(&job);
    if (job.status != MAK_OK) MAK_FAIL(job.status, job.err);
    return job.cs;
  }
};

// One worker slot: a context and a stream, kept between requests.  The
// context's workspace is sized for the largest request it has served (its
// estimate is what the scheduler charges the slot with) and is given back
// when a much smaller request comes or when the scheduler asks for it.
struct SlotExec {
  int device = 0;
  mak_options opt{};
  PassBatcher* batcher = nullptr;
  hipStream_t st = nullptr;
  mak_ctx* ctx = nullptr;
  int64_t ctx_est = 0;  // estimate of the largest request the context has served

  SlotExec(int dev, const mak_options& o, PassBatcher* pb) : device(dev), opt(o), batcher(pb) {
    (void)hipSetDevice(device);
    (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  }
  ~SlotExec() {
    (void)hipSetDevice(device);
    release();
    if (st) (void)hipStreamDestroy(st);
  }
  // What the slot holds after serving a request of estimate est when it held
  // `held`: a request under half the held size gets a fresh workspace.
  static size_t hold_after(size_t est, size_t held) {
    if (held > 0 && est * 2 < held) return est;
    return est > held ? est : held;
  }
  void release() {
    if (ctx) {
      (void)hipSetDevice(device);
      (void)hipStreamSynchronize(st);
      mak_destroy(ctx);
    }
    ctx = nullptr;
    ctx_est = 0;
  }
  int run(SolveArgs& a, std::string& err, int64_t est) {
    (void)hipSetDevice(device);
    if (ctx && size_t(hold_after(size_t(est), size_t(ctx_est))) < size_t(ctx_est)) release();
    if (!ctx) {
      if (mak_create(&ctx, device, &opt) != MAK_OK) {
        ctx = nullptr;
        err = "context creation failed";
        return MAK_EHIP;
      }
      mak::set_pass_runner(ctx, batcher);
      ctx_est = 0;
    }
    ctx_est = int64_t(hold_after(size_t(est), size_t(ctx_est)));
    const mak_status s = mak_solve(ctx, a.points, a.N, a.L, a.tol, a.psi, a.cent, a.disp, &a.info, st);
    if (s != MAK_OK) err = mak_last_error(ctx);
    return s;
  }
};

using Scheduler = mak::sched::RequestScheduler<SolveArgs, SlotExec>;

}  // namespace

struct mak_server {
  mak_options opt{};
  PassBatcher batcher;
  std::unique_ptr<Scheduler> sched;
  std::mutex err_mu;
  std::string err;
};

extern "C" {

mak_status mak_server_create(mak_server** out, int device, const mak_options* opt,
                             size_t mem_budget_bytes, int32_t max_slots) {
  if (!out || max_slots < 1 || max_slots > 64) return MAK_EINVAL;
  if (opt && (opt->batch_window_us < 0 || opt->batch_window_us > 1000000)) return MAK_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return MAK_EHIP;
  }
  mak_server* s = new mak_server();
  mak_default_options(&s->opt);
  if (opt) s->opt = *opt;
  s->batcher.start(device, s->opt.precision);
  const mak_options o = s->opt;
  PassBatcher* pb = &s->batcher;
  s->sched = std::make_unique<Scheduler>(mem_budget_bytes, max_slots, [device, o, pb](int32_t) {
    return std::make_unique<SlotExec>(device, o, pb);
  });
  if (o.batch_window_us > 0) {
    Scheduler* sc = s->sched.get();
    s->batcher.b.configure(o.batch_window_us, [sc] { return int(sc->stats().active); });
  }
  *out = s;
  return MAK_OK;
}

mak_status mak_server_submit(mak_server* s, const double* points, int64_t N, double L, double tol,
                             double* psi, double* centroids, double* displacements, int64_t* req_id) {
  if (!s || !points || !psi || !centroids || !displacements || !req_id || N < 1 || !(L > 0) ||
      !(tol > 0))
    return MAK_EINVAL;
  SolveArgs a;
  a.points = points;
  a.N = N;
  a.L = L;
  a.tol = tol;
  a.psi = psi;
  a.cent = centroids;
  a.disp = displacements;
  std::string err;
  const int64_t id = s->sched->submit(a, mak_solve_memory_estimate(N, s->opt.precision), &err);
  if (id < 0) {
    std::lock_guard<std::mutex> lk(s->err_mu);
    s->err = err;
    return MAK_ENOMEM;
  }
  *req_id = id;
  return MAK_OK;
}

static void copy_out(const mak::sched::Ticket<SolveArgs>& t, mak_solve_info* info, double* times) {
  if (times) {
    times[0] = t.t_submit;
    times[1] = t.t_start;
    times[2] = t.t_end;
  }
  if (info && t.done) *info = t.payload.info;
}

mak_status mak_server_poll(mak_server* s, int64_t req_id, int32_t* done, mak_solve_info* info,
                           double* times) {
  if (!s || !done) return MAK_EINVAL;
  mak::sched::Ticket<SolveArgs> t;
  if (!s->sched->poll(req_id, &t)) return MAK_ENOTFOUND;
  *done = t.done ? 1 : 0;
  copy_out(t, info, times);
  return t.done ? mak_status(t.status) : MAK_OK;
}

mak_status mak_server_wait(mak_server* s, int64_t req_id, mak_solve_info* info, double* times) {
  if (!s) return MAK_EINVAL;
  mak::sched::Ticket<SolveArgs> t;
  if (!s->sched->wait(req_id, &t)) return MAK_ENOTFOUND;
  copy_out(t, info, times);
  if (t.status != MAK_OK) {
    std::lock_guard<std::mutex> lk(s->err_mu);
    s->err = t.err;
  }
  return mak_status(t.status);
}

mak_status mak_server_release(mak_server* s, int64_t req_id) {
  if (!s) return MAK_EINVAL;
  const int r = s->sched->release(req_id);
  return r == 0 ? MAK_OK : (r == 1 ? MAK_ENOTFOUND : MAK_EINVAL);
}

mak_status mak_server_stats(mak_server* s, mak_server_info* out) {
  if (!s || !out) return MAK_EINVAL;
  const mak::sched::Stats st = s->sched->stats();
  std::memset(out, 0, sizeof(*out));
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->queued = st.queued;
  out->active = st.active;
  out->peak_active = st.peak_active;
  out->admitted_while_busy = st.admitted_while_busy;
  out->used_bytes = st.used;
  out->peak_used_bytes = st.peak_used;
  out->budget_bytes = st.budget;
  out->releases = st.releases;
  s->batcher.b.counters(&out->pass_batches, &out->batched_passes, &out->max_batch);
  return MAK_OK;
}

const char* mak_server_last_error(const mak_server* s) { return s ? s->err.c_str() : ""; }

void mak_server_destroy(mak_server* s) {
  if (!s) return;
  s->sched->shutdown();  // finishes queued and running requests
  s->batcher.b.configure(0, {});
  s->sched.reset();
  s->batcher.b.stop();
  delete s;
}

}  // extern "C"
