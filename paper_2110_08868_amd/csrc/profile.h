// Opt-in kernel timing: HIP events bracket the main kernels on the stream
// they are launched on; durations are resolved when the profile is read.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "common.h"

namespace mak {

// Entries of the profile's summed clip work counters (mak_profile_counters).
constexpr int kProfCounters = 48;

struct ProfAcc {
  int64_t launches = 0;
  double ms = 0.0;
  double units = 0.0;   // work items (cells, rows) processed
  double flops = 0.0;   // counted arithmetic (work counters), if enabled
  double bytes = 0.0;   // algorithmic HBM bytes
};

struct Profiler {
  bool timing = false;
  bool counting = false;
  bool cells_only = false;  // time only the cell-pass kernels (names starting "clip")
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double units, flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, ProfAcc> acc;
  double counters[kProfCounters] = {0};  // clip work counters summed over launches

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    MAK_HIP(hipEventCreate(&e));
    return e;
  }
  // Resolve every pending pair (waits for them).
  void resolve() {
    for (auto& p : pending) {
      MAK_HIP(hipEventSynchronize(p.b));
      float ms = 0.f;
      MAK_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      ProfAcc& a = acc[p.name];
      a.launches += 1;
      a.ms += ms;
      a.units += p.units;
      a.flops += p.flops;
      a.bytes += p.bytes;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void clear() {
    resolve();
    acc.clear();
    for (double& c : counters) c = 0.0;
  }
  ~Profiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Profiler of the ABI call in progress on this thread (NULL: disabled).
extern thread_local Profiler* g_prof;

// Scoped bracket: records the start event at construction, the stop event at
// stop(); work figures may be added before stop().
struct ProfScope {
  Profiler* p;
  std::string name;
  hipStream_t st;
  hipEvent_t a{};
  double units = 0, flops = 0, bytes = 0;
  bool open = false;
  ProfScope(const char* n, hipStream_t s, double u = 0, double by = 0)
      : p(g_prof), name(n), st(s), units(u), bytes(by) {
    if (p && p->timing && (!p->cells_only || name.compare(0, 4, "clip") == 0)) {
      a = p->take();
      MAK_HIP(hipEventRecord(a, st));
      open = true;
    }
  }
  void stop() {
    if (!open) return;
    hipEvent_t b = p->take();
    MAK_HIP(hipEventRecord(b, st));
    p->pending.push_back({name, a, b, units, flops, bytes});
    open = false;
  }
  ~ProfScope() {
    try {
      stop();
    } catch (...) {
    }
  }
};

}  // namespace mak
