// Optional per-kernel timing with HIP events on the launch stream.  When a
// context enables it, the runtime installs a Profiler for the duration of each
// call; the launch sites bracket selected kernels with event pairs, and the
// elapsed times are summed when the call has synchronised.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

enum { PROF_SCF_ACTIVE = 0, PROF_FFT_Z = 1, PROF_FFT_STRIDED = 2, PROF_KINDS = 3 };

struct Profiler {
  struct Pair {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pair> open;  // recorded, not yet read
  size_t used = 0;
  double total_ms[PROF_KINDS] = {0, 0, 0};
  long long launches[PROF_KINDS] = {0, 0, 0};
  unsigned mask = ~0u;  // kinds that are timed (each timed launch adds an event pair)
  int every = 1;         // time one launch in `every` of each kind
  long long seen[PROF_KINDS] = {0, 0, 0};

  hipEvent_t take() {
    if (used == pool.size()) {
      // timing only: no system-scope fence (its cache write-back would be timed)
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  // read every recorded pair (the stream must have passed them)
  void collect() {
    for (auto& p : open) {
      float ms = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        total_ms[p.kind] += ms;
        launches[p.kind] += 1;
      }
    }
    open.clear();
    used = 0;
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

extern thread_local Profiler* g_profiler;

struct ProfScope {
  Profiler* p;
  hipEvent_t b = nullptr;
  int kind;
  hipStream_t s;
  ProfScope(int k, hipStream_t st) : p(g_profiler), kind(k), s(st) {
    if (p && !((p->mask >> k) & 1u)) p = nullptr;
    if (p && p->every > 1 && (p->seen[k]++ % p->every) != 0) p = nullptr;
    if (!p) return;
    if (p->open.size() > 8192) p->collect();
    hipEvent_t a = p->take();
    b = p->take();
    if (!a || !b) {
      p = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
    p->open.push_back({a, b, kind});
  }
  ~ProfScope() {
    if (p) (void)hipEventRecord(b, s);
  }
};
