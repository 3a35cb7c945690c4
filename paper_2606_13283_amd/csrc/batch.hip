// Batched SCF driver: many independent snapshots solved together on one GPU.
//
// Every snapshot keeps its own context (fields, FFT plan, SCF state).  One SCF
// iteration of the whole batch is: one cooperative launch of the SCF kernel in
// which snapshot i owns a group of G_i co-resident blocks (steps 1-4 of the
// iteration, with group-local all-reduces), then, for each slot of the
// iteration's fixed step sequence, ONE launch that runs that step for every
// unconverged snapshot whatever its grid size (fft_batch.hip, scf.hip).  Each
// snapshot's blocks run exactly the code of its unbatched launch on the same
// tiles, and every global sum is taken in an order fixed by the snapshot's own
// grid, so results are bit-identical to unbatched solves.
//
// Iterations are captured in a HIP graph (K iterations per graph launch); the
// host polls the snapshots' done flags one launch behind, and when enough
// snapshots have converged it rebuilds the launch tables over the rest
// (compaction) so that converged snapshots cost nothing.  The schedule -- the
// block budget of the cooperative kernel and K -- is picked by an autotuner
// that times the candidates on the live solve (none of them changes a result
// bit) and caches the choice per batch shape.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/arche.h"
#include "arche_internal.h"

namespace {

__global__ void k_gather_done(ScfState* const* __restrict__ sts, int n, int* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = sts[i]->done;
}

struct Launch {
  int kind;  // STEP_FFT / STEP_WEIGHT / STEP_REAL_MIX
  int fft_kind, sign, mode;
  int njobs;
  unsigned nblocks;
  size_t jobs_off, bbeg_off;  // into the device table buffer
};
struct CoopLaunch {
  int nsys, nblocks;
  size_t args_off, gbeg_off;
};

struct Schedule {
  int blocks = 0;  // cooperative block budget
  int k = 0;       // iterations per graph launch
};
std::mutex g_tune_mtx;
std::map<std::string, Schedule> g_tuned;  // per batch shape, for the life of the process

}  // namespace

struct arche_batch {
  int n = 0;
  std::vector<arche_ctx*> ctx;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int cap = 0;  // co-resident blocks of the batched cooperative kernel
  Schedule forced, sched;
  std::string shape;
  int32_t info[6] = {0, 0, 0, 0, 0, 0};
  // launch tables over the active snapshots
  std::vector<int> active;
  std::vector<CoopLaunch> coop;
  std::vector<Launch> launches;
  char* dev = nullptr;
  size_t dev_cap = 0;
  ScfState** states_d = nullptr;
  int* done_d = nullptr;
  int* done_h = nullptr;  // pinned [2][n]
  DevAllocator dalloc_;   // the allocator installed when the batch was created
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_full = false;
  int graph_k = 0;
};

namespace {

arche_status berr(arche_batch* b, arche_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}
arche_status bhip(arche_batch* b, hipError_t e, const char* what) {
  (void)hipGetLastError();
  return berr(b, ARCHE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define BK(x)                                   \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return bhip(b, e_, #x); \
  } while (0)

void drop_graph(arche_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

struct HostTable {
  std::vector<char> buf;
  size_t put(const void* p, size_t bytes) {
    size_t off = (buf.size() + 255) & ~(size_t)255;
    buf.resize(off + bytes);
    std::memcpy(buf.data() + off, p, bytes);
    return off;
  }
};

// Launch tables over b->active with a cooperative budget of `budget` blocks.
arche_status build_tables(arche_batch* b, int budget) {
  HostTable t;
  b->coop.clear();
  b->launches.clear();
  budget = std::max(1, std::min(budget, b->cap));
  // cooperative groups: G_i proportional to the snapshot's chunks, at least 1,
  // at most its chunk count (and its context's flag array)
  int64_t tot = 0;
  for (int i : b->active) tot += b->ctx[i]->active.nchunk;
  std::vector<int> G;
  for (int i : b->active) {
    const arche_ctx* c = b->ctx[i];
    int64_t g = tot > 0 ? (int64_t)budget * c->active.nchunk / tot : 1;
    g = std::max<int64_t>(1, std::min<int64_t>(g, std::min<int64_t>(c->active.nchunk, c->coop_blocks)));
    G.push_back((int)g);
  }
  // split into cooperative launches of at most cap blocks each
  size_t q = 0;
  while (q < b->active.size()) {
    std::vector<ActiveArgs> args;
    std::vector<int> beg{0};
    while (q < b->active.size() && beg.back() + G[q] <= b->cap) {
      args.push_back(b->ctx[b->active[q]]->active);
      beg.push_back(beg.back() + G[q]);
      ++q;
    }
    if (args.empty()) return berr(b, ARCHE_EINVAL, "snapshot needs more blocks than one cooperative launch holds");
    CoopLaunch cl;
    cl.nsys = (int)args.size();
    cl.nblocks = beg.back();
    cl.args_off = t.put(args.data(), args.size() * sizeof(ActiveArgs));
    cl.gbeg_off = t.put(beg.data(), beg.size() * sizeof(int));
    b->coop.push_back(cl);
  }
  // one launch per slot over the snapshots that have the step
  for (int slot = 0; slot < SLOT_COUNT; ++slot) {
    std::vector<FftPass> fj;
    std::vector<MixWeightArgs> wj;
    std::vector<RealMixArgs> rj;
    std::vector<int> beg{0};
    Launch L{};
    L.kind = -1;
    for (int i : b->active) {
      for (const IterStep& st : b->ctx[i]->steps) {
        if (st.slot != slot) continue;
        if (L.kind < 0) {
          L.kind = st.kind;
          L.fft_kind = st.fft.kind;
          L.sign = st.fft.sign;
          L.mode = st.fft.mode;
        }
        if (st.kind != L.kind || (st.kind == STEP_FFT && (st.fft.kind != L.fft_kind || st.fft.sign != L.sign ||
                                                          st.fft.mode != L.mode)))
          return berr(b, ARCHE_EINVAL, "internal: inconsistent step slot");
        if (st.kind == STEP_FFT) fj.push_back(st.fft);
        if (st.kind == STEP_WEIGHT) wj.push_back(st.mw);
        if (st.kind == STEP_REAL_MIX) rj.push_back(st.rm);
        beg.push_back(beg.back() + (int)st.nblocks);
      }
    }
    if (L.kind < 0) continue;
    L.nblocks = (unsigned)beg.back();
    if (L.kind == STEP_FFT) {
      L.njobs = (int)fj.size();
      L.jobs_off = t.put(fj.data(), fj.size() * sizeof(FftPass));
    } else if (L.kind == STEP_WEIGHT) {
      L.njobs = (int)wj.size();
      L.jobs_off = t.put(wj.data(), wj.size() * sizeof(MixWeightArgs));
    } else {
      L.njobs = (int)rj.size();
      L.jobs_off = t.put(rj.data(), rj.size() * sizeof(RealMixArgs));
    }
    L.bbeg_off = t.put(beg.data(), beg.size() * sizeof(int));
    b->launches.push_back(L);
  }
  // the tables may be in use by queued work: wait, then replace them
  BK(hipStreamSynchronize(b->stream));
  drop_graph(b);
  if (t.buf.size() > b->dev_cap) {
    b->dalloc_.put(b->dev, b->stream);
    b->dev = nullptr;
    b->dev_cap = 0;
    BK(b->dalloc_.get((void**)&b->dev, t.buf.size(), b->stream));
    b->dev_cap = t.buf.size();
  }
  BK(hipMemcpy(b->dev, t.buf.data(), t.buf.size(), hipMemcpyHostToDevice));
  return ARCHE_OK;
}

hipError_t enqueue_coop(arche_batch* b) {
  for (const CoopLaunch& cl : b->coop) {
    hipError_t e = scf_active_batch_launch((const ActiveArgs*)(b->dev + cl.args_off), (const int*)(b->dev + cl.gbeg_off),
                                           cl.nsys, cl.nblocks, b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_passes(arche_batch* b) {
  for (const Launch& L : b->launches) {
    hipError_t e;
    const int* bbeg = (const int*)(b->dev + L.bbeg_off);
    if (L.kind == STEP_FFT)
      e = fft_batch_launch(L.fft_kind, L.sign, L.mode, (const FftPass*)(b->dev + L.jobs_off), bbeg, L.njobs, L.nblocks,
                           b->stream);
    else if (L.kind == STEP_WEIGHT)
      e = scf_weight_batch_launch((const MixWeightArgs*)(b->dev + L.jobs_off), L.njobs, b->stream);
    else
      e = scf_real_mix_batch_launch((const RealMixArgs*)(b->dev + L.jobs_off), bbeg, L.njobs, L.nblocks, b->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Capture K whole iterations; if the runtime cannot capture the cooperative
// launch, capture the passes of one iteration and launch the cooperative kernel
// before each replay instead.
arche_status build_graph(arche_batch* b, int k) {
  drop_graph(b);
  for (int full = 1; full >= 0; --full) {
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "hipStreamBeginCapture");
    const int kk = full ? k : 1;
    for (int it = 0; it < kk && e == hipSuccess; ++it) {
      if (full) e = enqueue_coop(b);
      if (e == hipSuccess) e = enqueue_passes(b);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e == hipSuccess && e2 == hipSuccess && g) {
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (e == hipSuccess) {
        b->graph = g;
        b->exec = x;
        b->graph_full = full != 0;
        b->graph_k = kk;
        return ARCHE_OK;
      }
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!full) return bhip(b, e != hipSuccess ? e : e2, "graph capture of the batched iteration");
  }
  return berr(b, ARCHE_EHIP, "graph capture failed");
}

// One graph launch (K iterations), then the done flags into done_h[slot].
hipError_t launch_round(arche_batch* b, int slot, hipEvent_t ev) {
  hipError_t e = hipSuccess;
  if (!b->graph_full) e = enqueue_coop(b);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather_done, dim3(1), dim3(256), 0, b->stream, (ScfState* const*)b->states_d, b->n, b->done_d);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->done_h + slot * b->n, b->done_d, b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipEventRecord(ev, b->stream);
  b->info[3]++;
  return e;
}

std::string shape_key(const arche_batch* b) {
  std::vector<int64_t> ng;
  for (const arche_ctx* c : b->ctx) ng.push_back(c->g.ng);
  std::sort(ng.begin(), ng.end());
  std::string s;
  for (int64_t v : ng) s += std::to_string(v) + ",";
  return s;
}

// Time `rounds` graph launches of the current tables/graph (seconds per iteration).
arche_status time_rounds(arche_batch* b, int rounds, hipEvent_t* ev, double* per_iter) {
  hipEvent_t t0, t1;
  BK(hipEventCreate(&t0));
  BK(hipEventCreate(&t1));
  BK(hipEventRecord(t0, b->stream));
  for (int r = 0; r < rounds; ++r) BK(launch_round(b, r & 1, ev[r & 1]));
  BK(hipEventRecord(t1, b->stream));
  BK(hipEventSynchronize(t1));
  float ms = 0.f;
  BK(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  *per_iter = 1e-3 * ms / (rounds * b->graph_k);
  return ARCHE_OK;
}

int count_active(const arche_batch* b, int slot) {
  int a = 0;
  for (int i : b->active) a += b->done_h[slot * b->n + i] == 0;
  return a;
}
void refresh_active(arche_batch* b, int slot) {
  std::vector<int> a;
  for (int i : b->active)
    if (b->done_h[slot * b->n + i] == 0) a.push_back(i);
  b->active.swap(a);
}

// The schedule: forced, cached for this shape, or measured now on the live solve.
arche_status choose_schedule(arche_batch* b, hipEvent_t* ev) {
  b->info[5] = 0;
  if (b->forced.blocks > 0 && b->forced.k > 0) {
    b->sched = b->forced;
    return ARCHE_OK;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mtx);
    auto it = g_tuned.find(b->shape);
    if (it != g_tuned.end()) {
      b->sched = it->second;
      if (b->forced.blocks > 0) b->sched.blocks = b->forced.blocks;
      if (b->forced.k > 0) b->sched.k = b->forced.k;
      return ARCHE_OK;
    }
  }
  b->info[5] = 1;
  Schedule best;
  double best_t = 1e30;
  std::vector<int> budgets;
  if (b->forced.blocks > 0)
    budgets.push_back(b->forced.blocks);
  else
    for (int d : {4, 2, 1}) budgets.push_back(std::max((int)b->active.size(), b->cap / d));
  for (int budget : budgets) {
    arche_status s = build_tables(b, budget);
    if (s == ARCHE_OK) s = build_graph(b, 1);
    double t = 0;
    if (s == ARCHE_OK) s = time_rounds(b, 2, ev, &t);
    if (s != ARCHE_OK) return s;
    if (t < best_t) {
      best_t = t;
      best.blocks = budget;
    }
  }
  // iterations per graph launch: more per launch saves launch gaps, costs up to
  // 2K idle iterations at the end; measured between 1 and 4
  best.k = 1;
  if (b->forced.k > 0) {
    best.k = b->forced.k;
  } else {
    arche_status s = build_tables(b, best.blocks);
    if (s == ARCHE_OK) s = build_graph(b, 4);
    double t4 = 0;
    if (s == ARCHE_OK) s = time_rounds(b, 1, ev, &t4);
    if (s != ARCHE_OK) return s;
    if (b->graph_full && t4 < 0.97 * best_t) best.k = 4;
  }
  b->sched = best;
  std::lock_guard<std::mutex> lk(g_tune_mtx);
  g_tuned[b->shape] = best;
  return ARCHE_OK;
}

arche_status batch_run(arche_batch* b) {
  hipEvent_t ev[2];
  BK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  BK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
  } guard{ev};
  b->active.clear();
  for (int i = 0; i < b->n; ++i) b->active.push_back(i);
  std::memset(b->done_h, 0, 2 * b->n * sizeof(int));
  b->info[3] = b->info[4] = 0;
  arche_status s = choose_schedule(b, ev);
  if (s != ARCHE_OK) return s;
  // tuning rounds (if any) have iterated: start from the device's view of done
  hipLaunchKernelGGL(k_gather_done, dim3(1), dim3(256), 0, b->stream, (ScfState* const*)b->states_d, b->n, b->done_d);
  BK(hipGetLastError());
  BK(hipMemcpyAsync(b->done_h, b->done_d, b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BK(hipStreamSynchronize(b->stream));
  refresh_active(b, 0);
  if (b->active.empty()) return ARCHE_OK;
  s = build_tables(b, b->sched.blocks);
  if (s == ARCHE_OK) s = build_graph(b, b->sched.k);
  if (s != ARCHE_OK) return s;
  b->info[0] = 0;
  for (const CoopLaunch& cl : b->coop) b->info[0] += cl.nblocks;
  b->info[1] = b->graph_k;
  b->info[2] = b->graph_full ? 1 : 0;
  int max_iter = 0;
  for (const arche_ctx* c : b->ctx) max_iter = std::max(max_iter, c->p.scf_max_iter);
  const int max_rounds = max_iter / std::max(1, b->graph_k) + 4;
  int table_size = (int)b->active.size();
  for (int r = 0; r < max_rounds; ++r) {
    BK(launch_round(b, r & 1, ev[r & 1]));
    if (r == 0) continue;
    const int prev = (r - 1) & 1;
    BK(hipEventSynchronize(ev[prev]));
    const int left = count_active(b, prev);
    if (left == 0) break;
    if (left <= (3 * table_size) / 4) {  // compaction
      refresh_active(b, prev);
      table_size = (int)b->active.size();
      s = build_tables(b, b->sched.blocks);
      if (s == ARCHE_OK) s = build_graph(b, b->sched.k);
      if (s != ARCHE_OK) return s;
      b->info[4]++;
    }
  }
  BK(hipStreamSynchronize(b->stream));
  return ARCHE_OK;
}

}  // namespace

extern "C" {

arche_status arche_batch_init(int32_t n_snap, const arche_params* p, void* hip_stream, arche_batch** out) {
  if (!out) return ARCHE_EINVAL;
  *out = nullptr;
  if (n_snap < 1 || !p) return ARCHE_EINVAL;
  arche_batch* b = new (std::nothrow) arche_batch();
  if (!b) return ARCHE_ENOMEM;
  auto fail = [&](arche_status s) {
    arche_batch_free(b);
    return s;
  };
  b->n = n_snap;
  b->dalloc_ = current_allocator();
  for (int i = 0; i < n_snap; ++i)
    for (int a = 0; a < 3; ++a)
      if (!fft_batch_supported(p[i].grid[a])) return fail(ARCHE_EINVAL);
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return fail(ARCHE_EHIP);
    b->own_stream = true;
  }
  for (int i = 0; i < n_snap; ++i) {
    arche_ctx* c = nullptr;
    arche_status s = arche_scf_init(&p[i], (void*)b->stream, &c);
    if (s != ARCHE_OK) return fail(s);
    b->ctx.push_back(c);
    scf_build_iteration(c);
    if (!c->fused) return fail(ARCHE_EINVAL);
  }
  b->cap = scf_batch_capacity();
  if (b->cap < 1) return fail(ARCHE_EHIP);
  std::vector<ScfState*> sts;
  for (arche_ctx* c : b->ctx) sts.push_back(c->state);
  if (b->dalloc_.get((void**)&b->states_d, n_snap * sizeof(ScfState*), b->stream) != hipSuccess)
    return fail(ARCHE_ENOMEM);
  if (b->dalloc_.get((void**)&b->done_d, n_snap * sizeof(int), b->stream) != hipSuccess) return fail(ARCHE_ENOMEM);
  if (hipHostMalloc((void**)&b->done_h, 2 * n_snap * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return fail(ARCHE_ENOMEM);
  if (hipMemcpy(b->states_d, sts.data(), n_snap * sizeof(ScfState*), hipMemcpyHostToDevice) != hipSuccess)
    return fail(ARCHE_EHIP);
  b->shape = shape_key(b);
  *out = b;
  return ARCHE_OK;
}

arche_status arche_batch_solve(arche_batch* b, const double* const* pos_host, arche_result* out,
                               double* const* forces_host) {
  if (!b) return ARCHE_EINVAL;
  if (!pos_host || !out) return berr(b, ARCHE_EINVAL, "NULL argument");
  b->err.clear();
  for (int i = 0; i < b->n; ++i)
    if (!pos_host[i]) return berr(b, ARCHE_EINVAL, "NULL positions for snapshot " + std::to_string(i));
  std::vector<int> fb(b->n, 0);
  for (int i = 0; i < b->n; ++i) {
    arche_status s = solve_begin(b->ctx[i], pos_host[i], b->ctx[i]->p.init, &fb[i]);
    if (s != ARCHE_OK) return berr(b, s, "snapshot " + std::to_string(i) + ": " + arche_last_error(b->ctx[i]));
  }
  arche_status s = batch_run(b);
  if (s != ARCHE_OK) return s;
  bool all = true;
  for (int i = 0; i < b->n; ++i) {
    arche_ctx* c = b->ctx[i];
    s = solve_collect(c, &out[i]);
    if (s == ARCHE_OK || s == ARCHE_ENOCONV) s = solve_finish(c, &out[i], fb[i]);
    if (s == ARCHE_ENOCONV) {
      all = false;
      continue;
    }
    if (s != ARCHE_OK) return berr(b, s, "snapshot " + std::to_string(i) + ": " + arche_last_error(c));
    if (forces_host && forces_host[i]) {
      s = solve_forces(c);
      if (s != ARCHE_OK) return berr(b, s, "snapshot " + std::to_string(i) + ": " + arche_last_error(c));
      std::memcpy(forces_host[i], c->h_forces.data(), 3 * c->n_atoms * sizeof(double));
    }
  }
  if (!all) return berr(b, ARCHE_ENOCONV, "some snapshots did not converge");
  return ARCHE_OK;
}

arche_ctx* arche_batch_context(arche_batch* b, int32_t i) {
  if (!b || i < 0 || i >= b->n) return nullptr;
  return b->ctx[i];
}

arche_status arche_batch_info(const arche_batch* b, int32_t info[6]) {
  if (!b || !info) return ARCHE_EINVAL;
  std::memcpy(info, b->info, sizeof(b->info));
  return ARCHE_OK;
}

arche_status arche_batch_set_schedule(arche_batch* b, int32_t coop_blocks, int32_t iters_per_graph) {
  if (!b || coop_blocks < 0 || iters_per_graph < 0 || iters_per_graph > 64) return ARCHE_EINVAL;
  b->forced.blocks = coop_blocks;
  b->forced.k = iters_per_graph;
  return ARCHE_OK;
}

const char* arche_batch_last_error(const arche_batch* b) { return b ? b->err.c_str() : ""; }

void arche_batch_free(arche_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (arche_ctx* c : b->ctx) arche_scf_free(c);
  b->dalloc_.put(b->dev, b->stream);
  b->dalloc_.put(b->states_d, b->stream);
  b->dalloc_.put(b->done_d, b->stream);
  if (b->done_h) (void)hipHostFree(b->done_h);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

arche_status arche_scf_solve_batch(int32_t n_snap, const arche_params* p, const double* const* pos_host,
                                   arche_result* out, void* hip_stream) {
  arche_batch* b = nullptr;
  arche_status s = arche_batch_init(n_snap, p, hip_stream, &b);
  if (s != ARCHE_OK) return s;
  s = arche_batch_solve(b, pos_host, out, nullptr);
  arche_batch_free(b);
  return s;
}

}  // extern "C"
