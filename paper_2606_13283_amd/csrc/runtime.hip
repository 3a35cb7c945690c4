// Host runtime behind the C ABI: context lifecycle, SCF driver loop, energies,
// pressure, forces and the Verlet MD step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/arche_kernels.h"
#include "arche_internal.h"

std::atomic<int> g_live_contexts{0};

namespace {

constexpr double PI = 3.14159265358979323846;
thread_local std::string g_init_err;

// ---- host evaluation of I_{1/2} (same coefficient tables as the device) ----
double fd_host(int j, double x) {
  if (x < FD_X_LO) {
    double y = std::exp(x), s = FD_SER[j][FD_KSER - 1];
    for (int k = FD_KSER - 2; k >= 0; --k) s = std::fma(s, y, FD_SER[j][k]);
    return y * s;
  }
  if (x >= FD_X_HI) {
    double u = 1.0 / (x * x), s = FD_ASY[j][FD_KASY - 1];
    for (int k = FD_KASY - 2; k >= 0; --k) s = std::fma(s, u, FD_ASY[j][k]);
    double r = std::sqrt(x);
    double p = (j == 0) ? 2.0 * r : (j == 1) ? x * r * (2.0 / 3.0) : x * x * r * 0.4;
    return p * std::fma(u, s, 1.0);
  }
  int i;
  const double t = fd_locate(x, i);
  double s = FD_POLY[j][i][FD_NCOEF - 1];
  for (int k = FD_NCOEF - 2; k >= 0; --k) s = std::fma(s, t, FD_POLY[j][i][k]);
  return s;
}

// X(y) = I_{1/2}^{-1}(y): Newton with a bisection safeguard on the monotone I_{1/2}
double fd_inverse_p12(double y) {
  double lo = std::log(y / 0.88622692545275801365) - 1e-9;  // I_{1/2}(x) < Gamma(3/2) e^x
  double hi = std::max(std::pow(1.5 * y, 2.0 / 3.0), lo + 1.0) + 1.0;
  while (fd_host(1, hi) < y) hi = 2.0 * hi + 1.0;
  while (fd_host(1, lo) > y) lo -= 1.0;
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    double f = fd_host(1, x) - y;
    if (f > 0) hi = x; else lo = x;
    double xn = x - f / (0.5 * fd_host(0, x));
    if (!(lo < xn && xn < hi)) xn = 0.5 * (lo + hi);
    if (std::fabs(xn - x) <= 2e-16 * std::max(1.0, std::fabs(x))) return xn;
    x = xn;
  }
  return x;
}

arche_status set_err(arche_ctx* c, arche_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

arche_status hip_err(arche_ctx* c, hipError_t e, const char* what) {
  return set_err(c, ARCHE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define CK(x)                                              \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return hip_err(c, e_, #x);       \
  } while (0)

template <class T>
hipError_t dalloc(arche_ctx* c, T** p, size_t n) {
  return c->dalloc_.get((void**)p, std::max<size_t>(n, 1) * sizeof(T), c->stream);
}

void free_all(arche_ctx* c) {
  void* ptrs[] = {c->ff_d, c->Vie, c->VH, c->lap_i, c->n_i, c->n_a, c->Vi, c->lap_a, c->rtmp, c->nhat_i, c->nhat_a, c->ctmp,
                  c->ctmp2, c->Sp, c->Sm, c->SZp, c->SZm, c->prev_nhat, c->prev_SZp, c->prev_SZm, c->shell_of,
                  c->shell_perm, c->shell_off, c->shell_g, c->pos, c->Zatom, c->forces, c->fpp, c->fpart, c->spec_d,
                  c->sp_order, c->sp_begin, c->Wp, c->Wm, c->phx, c->phy, c->phz, c->phT, c->partials, c->sums, c->state,
                  c->bar, c->err_d};
  for (void* p : ptrs) c->dalloc_.put(p, c->stream);
  if (c->state_host) (void)hipHostFree(c->state_host);
  if (c->iter_exec) (void)hipGraphExecDestroy(c->iter_exec);
  if (c->iter_graph) (void)hipGraphDestroy(c->iter_graph);
  c->iter_exec = nullptr;
  c->iter_graph = nullptr;
  delete c->prof;
  c->prof = nullptr;
  fft_plan_destroy_with(&c->plan, c->dalloc_.release, (void*)c->stream);
}

arche_status validate(const arche_params* p, std::string& msg) {
  if (!p) return msg = "params is NULL", ARCHE_EINVAL;
  if (p->n_atoms < 1) return msg = "n_atoms must be >= 1", ARCHE_EINVAL;
  if (p->n_species < 1 || p->n_species > ARCHE_MAX_SPECIES) return msg = "n_species must be in 1..8", ARCHE_EINVAL;
  if (!p->species || !p->Z || !p->rc || !p->mass) return msg = "species/Z/rc/mass arrays are required", ARCHE_EINVAL;
  for (int j = 0; j < p->n_atoms; ++j)
    if (p->species[j] < 0 || p->species[j] >= p->n_species) return msg = "species index out of range", ARCHE_EINVAL;
  for (int s = 0; s < p->n_species; ++s) {
    if (!(p->Z[s] > 0.0) || !std::isfinite(p->Z[s])) return msg = "Z must be positive", ARCHE_EINVAL;
    if (!(p->rc[s] >= 0.0) || !std::isfinite(p->rc[s])) return msg = "rc must be >= 0", ARCHE_EINVAL;
    if (!(p->mass[s] > 0.0) || !std::isfinite(p->mass[s])) return msg = "mass must be positive", ARCHE_EINVAL;
  }
  for (int a = 0; a < 3; ++a) {
    if (!(p->cell[a] > 0.0) || !std::isfinite(p->cell[a])) return msg = "cell edges must be positive", ARCHE_EINVAL;
    if (!fft_size_supported(p->grid[a]))
      return msg = "grid sizes must be even, <= 1024, with prime factors 2, 3, 5 only", ARCHE_EINVAL;
  }
  if (!(p->kT > 0.0) || !std::isfinite(p->kT)) return msg = "kT must be positive", ARCHE_EINVAL;
  if (!(p->lambda_vw >= 0.0) || !std::isfinite(p->lambda_vw)) return msg = "lambda_vw must be >= 0", ARCHE_EINVAL;
  if (p->xc != ARCHE_XC_NONE && p->xc != ARCHE_XC_LDA) return msg = "unknown xc", ARCHE_EINVAL;
  if (!(p->scf_tol > 0.0)) return msg = "scf_tol must be positive", ARCHE_EINVAL;
  if (p->scf_max_iter < 1) return msg = "scf_max_iter must be >= 1", ARCHE_EINVAL;
  if (p->mixing != ARCHE_MIX_FIXED && p->mixing != ARCHE_MIX_MORE && p->mixing != ARCHE_MIX_MORE_PRINTED)
    return msg = "unknown mixing", ARCHE_EINVAL;
  if (!(p->w_fixed >= 0.0 && p->w_fixed < 1.0)) return msg = "w_fixed must be in [0, 1)", ARCHE_EINVAL;
  if (p->more_warmup < 0) return msg = "more_warmup must be >= 0", ARCHE_EINVAL;
  if (!(p->more_trust > 0.0)) return msg = "more_trust must be positive", ARCHE_EINVAL;
  if (p->init < ARCHE_INIT_UNIFORM || p->init > ARCHE_INIT_LEARNED) return msg = "unknown init", ARCHE_EINVAL;
  if (!std::isfinite(p->ewald_alpha)) return msg = "ewald_alpha must be finite", ARCHE_EINVAL;
  if (p->ff_table) {
    if (p->ff_len < 4) return msg = "ff_len must be >= 4", ARCHE_EINVAL;
    if (!(p->ff_dq > 0.0) || !std::isfinite(p->ff_dq)) return msg = "ff_dq must be positive", ARCHE_EINVAL;
    for (int64_t i = 0; i < (int64_t)p->ff_len * p->n_species; ++i)
      if (!std::isfinite(p->ff_table[i])) return msg = "ff_table holds a non-finite value", ARCHE_EINVAL;
    // the cubic around the largest |k| of the box reads the node floor(q/dq) + 2
    double q2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double kn = (p->grid[a] / 2) / p->cell[a];
      q2 += kn * kn;
    }
    const double need = std::floor(std::sqrt(q2) / p->ff_dq) + 2.0;
    if (need > (double)(p->ff_len - 1))
      return msg = "ff_table does not reach two nodes past the largest |k| of the grid", ARCHE_EINVAL;
  }
  return ARCHE_OK;
}

// SCF state -> result fields and the context's error text
arche_status collect_state(arche_ctx* c, arche_result* out) {
  ScfState st;
  CK(hipMemcpyAsync(&st, c->state, sizeof(ScfState), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  std::memset(out, 0, sizeof(*out));
  out->mu = st.mu;
  out->residual = st.res;
  out->w_last = st.w;
  out->scf_iters = st.iter;
  out->newton_iters = st.newton_total;
  out->converged = st.done && !st.err && st.res < c->p.scf_tol;
  c->converged = out->converged;
  if (st.err) {
    c->err = st.mu_fail ? "chemical-potential search did not converge" : "non-finite value or barrier time-out in SCF";
  } else if (!out->converged) {
    c->err = "SCF did not reach scf_tol within scf_max_iter";
  }
  return ARCHE_OK;
}

// K whole iterations (the cooperative kernel and every pass) captured in one
// HIP graph, on grids whose passes all stop by themselves once the solve is done
// (so iterations past convergence cost only their launches).  Capture failure
// leaves the context on the launch-by-launch loop.
bool build_iteration_graph(arche_ctx* c) {
  c->graph_tried = true;
  scf_build_iteration(c);
  if (!c->fused) return false;
  const char* env = std::getenv("ARCHE_GRAPH");
  if (env && env[0] == '0') return false;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  hipError_t e = hipSuccess;
  for (int it = 0; it < ARCHE_GRAPH_ITERS && e == hipSuccess; ++it) e = scf_iteration(c);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (e == hipSuccess && e2 == hipSuccess && g) {
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) {
      c->iter_graph = g;
      c->iter_exec = x;
      c->graph_plain = scf_plain_launch(c);
      return true;
    }
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  return false;
}

// SCF loop.  Work is enqueued in units of ARCHE_GRAPH_ITERS iterations (a graph
// launch, or the iterations launch by launch when timing kernels; fewer for the
// tail below scf_max_iter), one unit ahead of the convergence poll: after
// enqueuing unit u the host waits for unit u-1 and reads its iterations' states
// from the pinned ring (the weight kernel of iteration t writes
// ring[(t-1) % ARCHE_RING]; two units fit).  Each unit boundary costs the device
// a few microseconds, so units of several iterations also when timing.  The state was reset by begin_solve; the iteration that meets the
// tolerance raises done and everything after it does nothing.  The polled states
// are kept as the solve's convergence history.
arche_status run_scf(arche_ctx* c, arche_result* out) {
  c->hist.clear();
  if (c->iter_exec && c->graph_plain != scf_plain_launch(c)) {
    // the launch mode of the SCF kernel changed (contexts came or went): capture again
    (void)hipGraphExecDestroy(c->iter_exec);
    (void)hipGraphDestroy(c->iter_graph);
    c->iter_exec = nullptr;
    c->iter_graph = nullptr;
    c->graph_tried = false;
  }
  if (!c->graph_tried && !c->prof) build_iteration_graph(c);
  const bool graph = c->iter_exec && !c->prof;
  hipEvent_t ev[2];
  CK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  CK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  const ScfState* ring = c->state_host;
  const int max_iter = c->p.scf_max_iter;
  bool stop = false;
  int launched = 0, read = 0, unit = 0;
  int unit_end[2] = {0, 0};
  // read the states of iterations read+1 .. upto from the ring
  auto consume = [&](int upto) {
    for (int j = read + 1; j <= upto && !stop; ++j) {
      const ScfState& s = ring[(j - 1) % ARCHE_RING];
      if (s.iter != j) {  // iteration j did nothing: the solve ended before it
        stop = true;
        break;
      }
      c->hist.push_back(s);
      read = j;
      if (s.done) stop = true;
    }
  };
  hipError_t e = hipSuccess;
  while (!stop && launched < max_iter && e == hipSuccess) {
    const int n = std::min(ARCHE_GRAPH_ITERS, max_iter - launched);
    if (graph && n == ARCHE_GRAPH_ITERS) {
      e = hipGraphLaunch(c->iter_exec, c->stream);
    } else {
      for (int i = 0; i < n && e == hipSuccess; ++i) e = scf_iteration(c);
    }
    launched += n;
    if (e == hipSuccess) e = hipEventRecord(ev[unit & 1], c->stream);
    unit_end[unit & 1] = launched;
    if (e == hipSuccess && unit >= 1) {
      e = hipEventSynchronize(ev[(unit - 1) & 1]);
      if (e == hipSuccess) consume(unit_end[(unit - 1) & 1]);
    }
    ++unit;
  }
  // the last unit (stopped by the iteration cap, or done inside it)
  if (e == hipSuccess && !stop && unit >= 1) {
    e = hipEventSynchronize(ev[(unit - 1) & 1]);
    if (e == hipSuccess) consume(unit_end[(unit - 1) & 1]);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (e != hipSuccess) return hip_err(c, e, "scf iteration");
  return collect_state(c, out);
}

arche_status evaluate(arche_ctx* c, arche_result* out) {
  double e[9];
  CK(scf_energies(c, e));
  const double alpha = ewald_alpha(c);
  double U3[3];
  CK(ionic_ewald(c, U3, alpha));
  double pie = 0.0;
  CK(ionic_pressure_ie(c, c->nhat_a, &pie));
  const GridInfo& g = c->g;
  double Ealpha = 0.0;
  for (int j = 0; j < c->n_atoms; ++j) {
    const int s = c->species[j];
    // lim_{q->0} [V_s(q) + Z_s/(pi q^2)]: 2 pi Z r_c^2 for the empty core, D_s(0) for a table
    Ealpha += c->ff_host.empty() ? 2.0 * PI * c->Z[s] * c->rc[s] * c->rc[s] : c->ff_host[(size_t)s * c->p.ff_len];
  }
  Ealpha *= c->Ne / g.vol;
  const double Eie = e[4] + Ealpha;
  const double Uii = U3[0] + U3[1] + U3[2];
  out->terms[ARCHE_T_FTF] = e[0];
  out->terms[ARCHE_T_KE] = e[1];
  out->terms[ARCHE_T_FVW] = e[7];
  out->terms[ARCHE_T_EH] = e[6];
  out->terms[ARCHE_T_FXC] = e[2];
  out->terms[ARCHE_T_EIE] = Eie;
  out->terms[ARCHE_T_UII] = Uii;
  out->terms[ARCHE_T_UPP] = U3[0];
  out->terms[ARCHE_T_UPM] = U3[1];
  out->terms[ARCHE_T_UJE] = U3[2];
  out->terms[ARCHE_T_ALPHA] = alpha;
  out->F = e[0] + e[7] + e[6] + e[2] + Eie + Uii;
  out->E = e[1] + e[7] + e[6] + e[2] + Eie + Uii;
  out->pterms[ARCHE_P_TF] = e[8];
  out->pterms[ARCHE_P_VW] = 2.0 * e[7] / (3.0 * g.vol);
  out->pterms[ARCHE_P_H] = e[6] / (3.0 * g.vol);
  out->pterms[ARCHE_P_XC] = e[3];
  out->pterms[ARCHE_P_IE] = Eie / g.vol + pie / (3.0 * g.vol * g.vol);
  out->pterms[ARCHE_P_II] = Uii / (3.0 * g.vol);
  out->P = 0.0;
  for (int k = 0; k < ARCHE_P_COUNT; ++k) out->P += out->pterms[k];
  return ARCHE_OK;
}

// installs the context's profiler (if enabled) for the duration of one call
struct ProfInstall {
  Profiler* p;
  explicit ProfInstall(arche_ctx* c) : p(c->prof) { g_profiler = p; }
  ~ProfInstall() {
    if (p) p->collect();
    g_profiler = nullptr;
  }
};

// positions, structure factor and ionic field, initial density, fresh SCF state
arche_status begin_solve(arche_ctx* c, const double* pos_host, int init, int* fallback) {
  const int n = c->n_atoms;
  for (int q = 0; q < 3 * n; ++q)
    if (!std::isfinite(pos_host[q])) return set_err(c, ARCHE_EINVAL, "non-finite position");
  c->err.clear();
  c->h_pos.assign(pos_host, pos_host + 3 * n);
  c->forces_ready = false;
  CK(hipMemcpyAsync(c->pos, c->h_pos.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  CK(ionic_structure(c));
  *fallback = 0;
  if (init == ARCHE_INIT_LEARNED && c->have_prev && c->init_net) {
    // plain guess -> n_i (one-center, or uniform when it rings negative); the
    // network's input G = n0 + (superposition change since the previous step)
    // in lap_a (free before the SCF); proposal from [G, previous converged n_a]
    // -> rtmp, floored and renormalised
    int plain_fb = 0;
    CK(scf_one_center_density(c, &plain_fb, nullptr, c->lap_a));
    CK(scf_add_scalar(c, c->lap_a, c->Ne / c->g.vol));
    CK(hipStreamSynchronize(c->stream));
    arche_status s = arche_net_forward(c->init_net, c->lap_a, c->n_a, c->Ne / c->g.vol, c->rtmp);
    if (s != ARCHE_OK) return set_err(c, s, std::string("learned guess: ") + arche_net_last_error(c->init_net));
    s = arche_net_sync(c->init_net);
    if (s != ARCHE_OK) return set_err(c, s, std::string("learned guess: ") + arche_net_last_error(c->init_net));
    CK(scf_learned_proposal(c));
    bool ok = false;
    CK(scf_floor_renorm(c, c->rtmp, &ok));
    if (ok) CK(hipMemcpyAsync(c->n_i, c->rtmp, c->g.ng * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    *fallback = ok ? 0 : 1;
    CK(scf_prepare_input(c));
  } else if ((init == ARCHE_INIT_ONE_CENTER || init == ARCHE_INIT_LEARNED) && c->have_prev) {
    CK(scf_initial_one_center(c, fallback));
    if (init == ARCHE_INIT_LEARNED) *fallback = 1;
  } else if (init == ARCHE_INIT_KEEP && c->solved) {
    CK(scf_prepare_input(c));
  } else {
    CK(scf_initial_uniform(c));
  }
  CK(scf_reset_state(c, NAN));
  return ARCHE_OK;
}

// energies and pressure at the converged state; keeps what the next guess needs
arche_status finish_solve(arche_ctx* c, arche_result* out, int fallback) {
  out->used_fallback = fallback;
  arche_status s = evaluate(c, out);
  if (s != ARCHE_OK) return s;
  // keep the converged spectrum and the charge structure factor for the next one-center guess
  const size_t hb = c->g.nh * sizeof(cplx);
  CK(hipMemcpyAsync(c->prev_nhat, c->nhat_a, hb, hipMemcpyDeviceToDevice, c->stream));
  CK(hipMemcpyAsync(c->prev_SZp, c->SZp, hb, hipMemcpyDeviceToDevice, c->stream));
  CK(hipMemcpyAsync(c->prev_SZm, c->SZm, hb, hipMemcpyDeviceToDevice, c->stream));
  CK(hipStreamSynchronize(c->stream));
  c->have_prev = out->converged;
  c->solved = true;
  c->last = *out;
  return out->converged ? ARCHE_OK : ARCHE_ENOCONV;
}

arche_status do_solve(arche_ctx* c, const double* pos_host, arche_result* out, int init) {
  ProfInstall pi(c);
  int fallback = 0;
  arche_status s = begin_solve(c, pos_host, init, &fallback);
  if (s != ARCHE_OK) return s;
  s = run_scf(c, out);
  if (s != ARCHE_OK) return s;
  return finish_solve(c, out, fallback);
}

arche_status do_forces(arche_ctx* c) {
  ProfInstall pi(c);
  if (!c->forces_ready) {
    CK(ionic_forces(c, c->nhat_a, c->forces));
    c->h_forces.resize(3 * c->n_atoms);
    CK(hipMemcpyAsync(c->h_forces.data(), c->forces, 3 * c->n_atoms * sizeof(double), hipMemcpyDeviceToHost,
                      c->stream));
    CK(hipStreamSynchronize(c->stream));
    c->forces_ready = true;
  }
  return ARCHE_OK;
}

}  // namespace

arche_status solve_begin(arche_ctx* c, const double* pos_host, int init, int* fallback) {
  return begin_solve(c, pos_host, init, fallback);
}
arche_status solve_collect(arche_ctx* c, arche_result* out) { return collect_state(c, out); }
arche_status solve_finish(arche_ctx* c, arche_result* out, int fallback) { return finish_solve(c, out, fallback); }
arche_status solve_forces(arche_ctx* c) { return do_forces(c); }
arche_status ctx_error(arche_ctx* c, arche_status s, const std::string& m) { return set_err(c, s, m); }

// Verlet (Sec. 2.1) with the forces of the context's converged solve at r:
// the start r(-dt) = r - v dt + F dt^2/(2m), and r(t+dt) = 2 r - r(t-dt) + F dt^2/m
// with the central-difference velocity v(t) = (r(t+dt) - r(t-dt)) / (2 dt).
void verlet_start(const arche_ctx* c, double dt, const double* r, const double* vel, double* r_prev) {
  const std::vector<double>& F = c->h_forces;
  for (int j = 0; j < c->n_atoms; ++j) {
    const double m = c->mass[c->species[j]];
    for (int a = 0; a < 3; ++a) r_prev[3 * j + a] = r[3 * j + a] - vel[3 * j + a] * dt + F[3 * j + a] * dt * dt / (2.0 * m);
  }
}
void verlet_next(const arche_ctx* c, double dt, const double* r, const double* r_prev, double* rn, double* v) {
  const std::vector<double>& F = c->h_forces;
  for (int j = 0; j < c->n_atoms; ++j) {
    const double m = c->mass[c->species[j]];
    for (int a = 0; a < 3; ++a) {
      const int q = 3 * j + a;
      rn[q] = 2.0 * r[q] - r_prev[q] + F[q] * dt * dt / m;
      if (v) v[q] = (rn[q] - r_prev[q]) / (2.0 * dt);
    }
  }
}

// host Fermi-Dirac integrals for other host code (the average atom)
double host_fd(int j, double x) { return fd_host(j, x); }
double host_fd_inverse_p12(double y) { return fd_inverse_p12(y); }

namespace {
std::mutex g_alloc_mtx;
DevAllocator g_allocator;  // installed by arche_set_allocator (null pair: hipMalloc)
}  // namespace

DevAllocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mtx);
  return g_allocator;
}

extern "C" {

arche_status arche_scf_init(const arche_params* p, void* hip_stream, arche_ctx** out) {
  if (!out) {
    g_init_err = "out is NULL";
    return ARCHE_EINVAL;
  }
  *out = nullptr;
  std::string msg;
  arche_status vs = validate(p, msg);
  if (vs != ARCHE_OK) {
    g_init_err = msg;
    return vs;
  }
  arche_ctx* c = new (std::nothrow) arche_ctx();
  if (!c) {
    g_init_err = "host allocation failed";
    return ARCHE_ENOMEM;
  }
  c->p = *p;
  c->p.species = nullptr;
  c->p.Z = c->p.rc = c->p.mass = nullptr;
  c->p.ff_table = nullptr;
  c->dalloc_ = current_allocator();
  if (p->ff_table) c->ff_host.assign(p->ff_table, p->ff_table + (size_t)p->ff_len * p->n_species);
  c->n_atoms = p->n_atoms;
  c->n_species = p->n_species;
  c->species.assign(p->species, p->species + p->n_atoms);
  c->Z.assign(p->Z, p->Z + p->n_species);
  c->rc.assign(p->rc, p->rc + p->n_species);
  c->mass.assign(p->mass, p->mass + p->n_species);
  c->Zj.resize(c->n_atoms);
  for (int j = 0; j < c->n_atoms; ++j) {
    c->Zj[j] = c->Z[c->species[j]];
    c->Ne += c->Zj[j];
    c->sumZ2 += c->Zj[j] * c->Zj[j];
  }
  c->Q = c->Ne;
  GridInfo& g = c->g;
  for (int a = 0; a < 3; ++a) {
    g.N[a] = p->grid[a];
    g.L[a] = p->cell[a];
  }
  g.Nh = g.N[2] / 2 + 1;
  g.ng = (int64_t)g.N[0] * g.N[1] * g.N[2];
  g.nh = (int64_t)g.N[0] * g.N[1] * g.Nh;
  g.vol = g.L[0] * g.L[1] * g.L[2];
  g.dv = g.vol / (double)g.ng;
  c->sp.ns = c->n_species;
  for (int s = 0; s < c->n_species; ++s) {
    c->sp.Z[s] = c->Z[s];
    c->sp.rc[s] = c->rc[s];
  }
  const double cn = std::pow(2.0 * p->kT, 1.5) / (2.0 * PI * PI);
  c->eta0 = fd_inverse_p12(c->Ne / g.vol / cn);

  auto fail_init = [&](arche_status s, const std::string& m) {
    g_init_err = m;
    free_all(c);
    if (c->stream && !hip_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return fail_init(ARCHE_EHIP, "no HIP device");
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    return fail_init(ARCHE_EHIP, "hipStreamCreate failed");
  } else {
    c->own_stream = true;
  }
  int dev_attr = 0;
  (void)hipDeviceGetAttribute(&dev_attr, hipDeviceAttributeCooperativeLaunch, c->device);
  if (!dev_attr) return fail_init(ARCHE_EHIP, "device does not support cooperative launches");
  if (!fft_plan_create_with(&c->plan, g.N, c->dalloc_.alloc, c->dalloc_.release, (void*)c->stream))
    return fail_init(ARCHE_ENOMEM, "FFT plan creation failed");
  c->fdt = fd_tables_device(c->device);
  if (!c->fdt) return fail_init(ARCHE_ENOMEM, "Fermi-Dirac table upload failed");
  c->coop_blocks = scf_coop_blocks(g.ng);
  if (c->coop_blocks < 1) return fail_init(ARCHE_EHIP, "cooperative occupancy query failed");

  const int ns = c->n_species, n = c->n_atoms;
  bool ok = true;
  for (double** f : {&c->Vie, &c->VH, &c->lap_i, &c->n_i, &c->n_a, &c->Vi, &c->lap_a, &c->rtmp})
    ok = ok && dalloc(c, f, g.ng) == hipSuccess;
  for (cplx** f : {&c->nhat_i, &c->nhat_a, &c->ctmp, &c->ctmp2, &c->SZp, &c->SZm, &c->prev_nhat, &c->prev_SZp,
                   &c->prev_SZm})
    ok = ok && dalloc(c, f, g.nh) == hipSuccess;
  for (cplx** f : {&c->Sp, &c->Sm, &c->Wp, &c->Wm}) ok = ok && dalloc(c, f, (size_t)ns * g.nh) == hipSuccess;
  ok = ok && dalloc(c, &c->phx, (size_t)n * g.N[0]) == hipSuccess;
  ok = ok && dalloc(c, &c->phy, (size_t)n * g.N[1]) == hipSuccess;
  ok = ok && dalloc(c, &c->phz, (size_t)n * g.Nh) == hipSuccess;
  ok = ok && dalloc(c, &c->phT, (size_t)n * (g.N[0] + g.N[1] + g.Nh)) == hipSuccess;
  ok = ok && dalloc(c, &c->pos, 3 * (size_t)n) == hipSuccess;
  ok = ok && dalloc(c, &c->Zatom, (size_t)n) == hipSuccess;
  ok = ok && dalloc(c, &c->forces, 3 * (size_t)n) == hipSuccess;
  ok = ok && dalloc(c, &c->fpp, 3 * (size_t)n) == hipSuccess;
  ok = ok && dalloc(c, &c->spec_d, (size_t)n) == hipSuccess;
  ok = ok && dalloc(c, &c->sp_order, (size_t)n) == hipSuccess;
  ok = ok && dalloc(c, &c->sp_begin, (size_t)ns + 1) == hipSuccess;
  c->partial_cap = (int)scf_part_offset(c) + 64 * 1024 + 7 * n + 64;
  ok = ok && dalloc(c, &c->partials, (size_t)c->partial_cap) == hipSuccess;
  ok = ok && dalloc(c, &c->sums, 64) == hipSuccess;
  ok = ok && dalloc(c, &c->state, 1) == hipSuccess;
  ok = ok && dalloc(c, &c->bar, (size_t)SCF_BAR_WORDS) == hipSuccess;
  ok = ok && dalloc(c, &c->err_d, 1) == hipSuccess;
  if (ok) ok = dalloc(c, &c->fpart, ionic_force_partials(c)) == hipSuccess;
  if (ok && !c->ff_host.empty()) ok = dalloc(c, &c->ff_d, c->ff_host.size()) == hipSuccess;
  if (ok) ok = hipHostMalloc((void**)&c->state_host, ARCHE_RING * sizeof(ScfState), hipHostMallocDefault) == hipSuccess;
  if (!ok) return fail_init(ARCHE_ENOMEM, "device allocation failed");
  std::vector<int32_t> order(n), begin(ns + 1, 0);
  {
    int q = 0;
    for (int s = 0; s < ns; ++s) {
      begin[s] = q;
      for (int j = 0; j < n; ++j)
        if (c->species[j] == s) order[q++] = j;
    }
    begin[ns] = q;
  }
  bool up = hipMemcpy(c->Zatom, c->Zj.data(), n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->spec_d, c->species.data(), n * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->sp_order, order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(c->sp_begin, begin.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
            (c->ff_host.empty() || hipMemcpy(c->ff_d, c->ff_host.data(), c->ff_host.size() * sizeof(double),
                                             hipMemcpyHostToDevice) == hipSuccess);
  if (!up) return fail_init(ARCHE_EHIP, "upload failed");
  c->sp.ff = c->ff_d;
  c->sp.ff_len = c->ff_host.empty() ? 0 : p->ff_len;
  c->sp.ff_dq = c->ff_host.empty() ? 0.0 : p->ff_dq;
  if (ionic_shells(c) != hipSuccess) return fail_init(ARCHE_ENOMEM, "shell table allocation failed");
  if (fft_tune(&c->plan, c->ctmp, c->rtmp, c->stream) != hipSuccess) return fail_init(ARCHE_EHIP, "FFT tile tuning failed");
  g_live_contexts.fetch_add(1);
  *out = c;
  return ARCHE_OK;
}

arche_status arche_scf_solve(arche_ctx* c, const double* pos_host, arche_result* out) {
  if (!c || !pos_host || !out) return set_err(c, ARCHE_EINVAL, "NULL argument");
  return do_solve(c, pos_host, out, c->p.init);
}

arche_status arche_forces(arche_ctx* c, double* forces_host) {
  if (!c || !forces_host) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!c->solved || !c->converged) return set_err(c, ARCHE_ESTATE, "no converged solve");
  arche_status s = do_forces(c);
  if (s != ARCHE_OK) return s;
  std::memcpy(forces_host, c->h_forces.data(), 3 * c->n_atoms * sizeof(double));
  return ARCHE_OK;
}

arche_status arche_md_step(arche_ctx* c, double dt, double* pos_io, double* vel_io, double* forces_out,
                           arche_result* out) {
  if (!c || !pos_io || !vel_io || !out) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(c, ARCHE_EINVAL, "dt must be positive");
  const int n = c->n_atoms;
  for (int q = 0; q < 3 * n; ++q)
    if (!std::isfinite(pos_io[q]) || !std::isfinite(vel_io[q])) return set_err(c, ARCHE_EINVAL, "non-finite input");
  const bool same = c->solved && c->converged && c->h_pos.size() == (size_t)3 * n &&
                    std::memcmp(c->h_pos.data(), pos_io, 3 * n * sizeof(double)) == 0;
  if (!same) {
    c->have_r_prev = false;
    arche_result tmp;
    arche_status s = do_solve(c, pos_io, &tmp, c->p.init);
    if (s != ARCHE_OK) return s;
  }
  arche_status s = do_forces(c);
  if (s != ARCHE_OK) return s;
  std::vector<double> r(pos_io, pos_io + 3 * n), rn(3 * n), v(3 * n);
  if (!c->have_r_prev) {
    c->r_prev.resize(3 * n);
    verlet_start(c, dt, pos_io, vel_io, c->r_prev.data());
  }
  verlet_next(c, dt, pos_io, c->r_prev.data(), rn.data(), v.data());
  s = do_solve(c, rn.data(), out, c->p.init);
  if (s != ARCHE_OK) {
    c->have_r_prev = false;
    return s;
  }
  c->r_prev = r;
  c->have_r_prev = true;
  s = do_forces(c);
  if (s != ARCHE_OK) return s;
  std::memcpy(pos_io, rn.data(), 3 * n * sizeof(double));
  std::memcpy(vel_io, v.data(), 3 * n * sizeof(double));
  if (forces_out) std::memcpy(forces_out, c->h_forces.data(), 3 * n * sizeof(double));
  return ARCHE_OK;
}

arche_status arche_get_density(arche_ctx* c, double* dst, int32_t on_device) {
  if (!c || !dst) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!c->solved) return set_err(c, ARCHE_ESTATE, "no solve yet");
  CK(hipMemcpyAsync(dst, c->n_a, c->g.ng * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                    c->stream));
  CK(hipStreamSynchronize(c->stream));
  return ARCHE_OK;
}

arche_status arche_set_density(arche_ctx* c, const double* src, int32_t on_device) {
  if (!c || !src) return set_err(c, ARCHE_EINVAL, "NULL argument");
  const GridInfo& g = c->g;
  std::vector<double> h;
  if (on_device) {
    h.resize(g.ng);
    CK(hipMemcpy(h.data(), src, g.ng * sizeof(double), hipMemcpyDeviceToHost));
    src = h.data();
  }
  double tot = 0.0;
  for (int64_t i = 0; i < g.ng; ++i) {
    if (!(src[i] > 0.0) || !std::isfinite(src[i])) return set_err(c, ARCHE_EINVAL, "density must be positive");
    tot += src[i];
  }
  const double s = c->Ne / (tot * g.dv);
  std::vector<double> n(src, src + g.ng);
  for (auto& v : n) v *= s;
  CK(hipMemcpyAsync(c->n_i, n.data(), g.ng * sizeof(double), hipMemcpyHostToDevice, c->stream));
  CK(hipStreamSynchronize(c->stream));
  c->solved = true;  // an input density exists for ARCHE_INIT_KEEP
  c->converged = false;
  return ARCHE_OK;
}

arche_status arche_set_init_net(arche_ctx* c, arche_net* net) {
  if (!c) return ARCHE_EINVAL;
  c->init_net = net;
  return ARCHE_OK;
}

arche_status arche_reset_history(arche_ctx* c) {
  if (!c) return ARCHE_EINVAL;
  c->have_prev = false;
  c->have_r_prev = false;
  return ARCHE_OK;
}

arche_status arche_set_allocator(void* (*alloc)(size_t, void*), void (*release)(void*, void*)) {
  if ((alloc == nullptr) != (release == nullptr)) return ARCHE_EINVAL;
  std::lock_guard<std::mutex> lk(g_alloc_mtx);
  g_allocator.alloc = alloc;
  g_allocator.release = release;
  return ARCHE_OK;
}

void arche_scf_free(arche_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  g_live_contexts.fetch_sub(1);
}

arche_status arche_stress(arche_ctx* c, const double* vel_host, double* sigma_host, double* terms_host) {
  if (!c || !sigma_host) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!c->solved || !c->converged) return set_err(c, ARCHE_ESTATE, "no converged solve");
  ProfInstall pi(c);
  const GridInfo& g = c->g;
  const double V = g.vol, V2 = V * V;
  const double alpha = ewald_alpha(c);
  const cplx* shat = nullptr;
  if (c->p.lambda_vw != 0.0) {
    CK(scf_sqrt_spectrum(c, c->n_a, c->ctmp));
    shat = c->ctmp;
  }
  double t[24], pp[6];
  CK(ionic_stress_sums(c, c->nhat_a, shat, alpha, t, pp));
  const arche_result& r = c->last;
  // per term, six components xx, yy, zz, yz, xz, xy
  double T[ARCHE_S_COUNT][6] = {};
  if (vel_host) {
    for (int j = 0; j < c->n_atoms; ++j) {
      const double m = c->mass[c->species[j]];
      const double* v = vel_host + 3 * j;
      const double vv[6] = {v[0] * v[0], v[1] * v[1], v[2] * v[2], v[1] * v[2], v[0] * v[2], v[0] * v[1]};
      for (int q = 0; q < 6; ++q) T[ARCHE_S_KIN][q] -= m * vv[q] / V;
    }
  }
  const double Upm_k = r.terms[ARCHE_T_UPM] + alpha / std::sqrt(PI) * c->sumZ2;  // (1/2V) sum V_a |S_Z|^2
  for (int q = 0; q < 6; ++q) {
    const double d = q < 3 ? 1.0 : 0.0;
    T[ARCHE_S_TF][q] = -r.pterms[ARCHE_P_TF] * d;
    T[ARCHE_S_XC][q] = -r.pterms[ARCHE_P_XC] * d;
    T[ARCHE_S_VW][q] = -c->p.lambda_vw * 4.0 * PI * PI / V2 * t[6 + q];
    T[ARCHE_S_EE][q] = t[q] / V2 - r.terms[ARCHE_T_EH] / V * d;
    T[ARCHE_S_IE][q] = -r.terms[ARCHE_T_EIE] / V * d - t[12 + q] / V2;
    T[ARCHE_S_II][q] = -pp[q] / V + t[18 + q] / V2 - Upm_k / V * d +
                       PI * c->Q * c->Q / (2.0 * alpha * alpha * V2) * d;
  }
  static const int row[6] = {0, 1, 2, 1, 0, 0}, col[6] = {0, 1, 2, 2, 2, 1};
  for (int a = 0; a < 9; ++a) sigma_host[a] = 0.0;
  for (int k = 0; k < ARCHE_S_COUNT; ++k) {
    double full[9];
    for (int q = 0; q < 6; ++q) full[3 * row[q] + col[q]] = full[3 * col[q] + row[q]] = T[k][q];
    for (int a = 0; a < 9; ++a) sigma_host[a] += full[a];
    if (terms_host)
      for (int a = 0; a < 9; ++a) terms_host[9 * k + a] = full[a];
  }
  return ARCHE_OK;
}

const char* arche_last_error(const arche_ctx* c) { return c ? c->err.c_str() : g_init_err.c_str(); }

const char* arche_version(void) { return "arche-mi355x 0.1 (gfx950, FP64)"; }

arche_status arche_debug_get(arche_ctx* c, int32_t which, double* dst_host) {
  if (!c || !dst_host) return set_err(c, ARCHE_EINVAL, "NULL argument");
  const GridInfo& g = c->g;
  const void* src = nullptr;
  size_t bytes = 0;
  switch (which) {
    case ARCHE_DBG_VIE: src = c->Vie; bytes = g.ng * sizeof(double); break;
    case ARCHE_DBG_VI: src = c->Vi; bytes = g.ng * sizeof(double); break;
    case ARCHE_DBG_NA: src = c->n_a; bytes = g.ng * sizeof(double); break;
    case ARCHE_DBG_NI: src = c->n_i; bytes = g.ng * sizeof(double); break;
    case ARCHE_DBG_SZP: src = c->SZp; bytes = g.nh * sizeof(cplx); break;
    case ARCHE_DBG_SZM: src = c->SZm; bytes = g.nh * sizeof(cplx); break;
    case ARCHE_DBG_NHAT_A: src = c->nhat_a; bytes = g.nh * sizeof(cplx); break;
    case ARCHE_DBG_FPP: src = c->fpp; bytes = 3 * c->n_atoms * sizeof(double); break;
    default: return set_err(c, ARCHE_EINVAL, "unknown debug field");
  }
  CK(hipMemcpyAsync(dst_host, src, bytes, hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  return ARCHE_OK;
}

arche_status arche_debug_one_center(arche_ctx* c, const double* pos_host, double* n_init_host, int32_t* used_fallback) {
  return arche_debug_one_center2(c, pos_host, n_init_host, used_fallback, nullptr);
}

arche_status arche_md_predict(arche_ctx* c, double dt, const double* pos_host, const double* vel_host,
                              double* next_host) {
  if (!c || !pos_host || !vel_host || !next_host) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_err(c, ARCHE_EINVAL, "dt must be positive");
  const int n = c->n_atoms;
  const bool same = c->solved && c->converged && c->h_pos.size() == (size_t)3 * n &&
                    std::memcmp(c->h_pos.data(), pos_host, 3 * n * sizeof(double)) == 0;
  if (!same) return set_err(c, ARCHE_ESTATE, "no converged solve at these positions");
  arche_status s = do_forces(c);
  if (s != ARCHE_OK) return s;
  std::vector<double> rp(3 * n);
  if (c->have_r_prev)
    rp = c->r_prev;
  else
    verlet_start(c, dt, pos_host, vel_host, rp.data());
  verlet_next(c, dt, pos_host, rp.data(), next_host, nullptr);
  return ARCHE_OK;
}

arche_status arche_learned_guide(arche_ctx* c, const double* next_pos_host, double* guide_host) {
  if (!c || !next_pos_host || !guide_host) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!c->have_prev || !c->solved || !c->converged) return set_err(c, ARCHE_ESTATE, "no converged previous step");
  for (int q = 0; q < 3 * c->n_atoms; ++q)
    if (!std::isfinite(next_pos_host[q])) return set_err(c, ARCHE_EINVAL, "non-finite position");
  // the ionic field and structure factors of the next positions (recomputed by
  // the next solve anyway); the converged state, its positions and forces stay
  CK(hipMemcpyAsync(c->pos, next_pos_host, 3 * c->n_atoms * sizeof(double), hipMemcpyHostToDevice, c->stream));
  CK(ionic_structure(c));
  int fb = 0;
  CK(scf_one_center_density(c, &fb, nullptr, c->lap_a));
  CK(scf_add_scalar(c, c->lap_a, c->Ne / c->g.vol));
  CK(hipMemcpyAsync(guide_host, c->lap_a, c->g.ng * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  // the device copy of the positions back to those of the converged solve
  CK(hipMemcpyAsync(c->pos, c->h_pos.data(), 3 * c->n_atoms * sizeof(double), hipMemcpyHostToDevice, c->stream));
  CK(ionic_structure(c));
  CK(hipStreamSynchronize(c->stream));
  return ARCHE_OK;
}

arche_status arche_debug_one_center2(arche_ctx* c, const double* pos_host, double* n_init_host, int32_t* used_fallback,
                                     double* raw_host) {
  if (!c || !pos_host || !n_init_host) return set_err(c, ARCHE_EINVAL, "NULL argument");
  if (!c->have_prev) return set_err(c, ARCHE_ESTATE, "no previous converged step");
  c->h_pos.assign(pos_host, pos_host + 3 * c->n_atoms);
  CK(hipMemcpyAsync(c->pos, pos_host, 3 * c->n_atoms * sizeof(double), hipMemcpyHostToDevice, c->stream));
  CK(ionic_structure(c));
  int fb = 0;
  CK(scf_one_center_density(c, &fb, nullptr, c->lap_a));
  CK(scf_add_scalar(c, c->lap_a, c->Ne / c->g.vol));
  CK(scf_prepare_input(c));
  if (used_fallback) *used_fallback = fb;
  if (raw_host) CK(hipMemcpyAsync(raw_host, c->lap_a, c->g.ng * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CK(hipMemcpyAsync(n_init_host, c->n_i, c->g.ng * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CK(hipStreamSynchronize(c->stream));
  c->solved = false;
  c->converged = false;
  return ARCHE_OK;
}

int32_t arche_debug_live_contexts(void) { return g_live_contexts.load(); }

arche_status arche_debug_history(arche_ctx* c, double* rows_host, int32_t max_rows, int32_t* n_rows) {
  if (!c || !n_rows) return ARCHE_EINVAL;
  const int n = (int)c->hist.size();
  *n_rows = n;
  if (!rows_host) return ARCHE_OK;
  for (int i = 0; i < n && i < max_rows; ++i) {
    const ScfState& s = c->hist[i];
    double* r = rows_host + 10 * (size_t)i;
    r[0] = s.iter;
    r[1] = s.res;
    r[2] = s.w;
    r[3] = s.mu;
    r[4] = s.K;
    r[5] = s.UH + s.Uxc + s.Uvw;
    r[6] = s.maxrel;
    r[7] = s.newton_last;
    r[8] = s.more_on;
    r[9] = s.err;
  }
  return ARCHE_OK;
}

arche_status arche_profile_enable(arche_ctx* c, int32_t on) {
  if (!c) return ARCHE_EINVAL;
  if (on && !c->prof) c->prof = new (std::nothrow) Profiler();
  if (on && !c->prof) return set_err(c, ARCHE_ENOMEM, "profiler allocation failed");
  if (on) {
    c->prof->mask = on == 1 ? ~0u : (unsigned)on >> 1;
    c->prof->every = 1;  // every launch of the timed kinds until arche_profile_sample
  }
  if (!on) {
    delete c->prof;
    c->prof = nullptr;
  }
  return ARCHE_OK;
}

arche_status arche_profile_sample(arche_ctx* c, int32_t every) {
  if (!c || every < 1) return ARCHE_EINVAL;
  if (!c->prof) return set_err(c, ARCHE_ESTATE, "profiling is not enabled");
  c->prof->every = every;
  return ARCHE_OK;
}

arche_status arche_profile_read(arche_ctx* c, int32_t kind, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches || kind < 0 || kind >= PROF_KINDS) return ARCHE_EINVAL;
  if (!c->prof) return set_err(c, ARCHE_ESTATE, "profiling is not enabled");
  *total_ms = c->prof->total_ms[kind];
  *launches = c->prof->launches[kind];
  return ARCHE_OK;
}

arche_status arche_profile_reset(arche_ctx* c) {
  if (!c) return ARCHE_EINVAL;
  if (c->prof) {
    for (int k = 0; k < PROF_KINDS; ++k) {
      c->prof->total_ms[k] = 0.0;
      c->prof->launches[k] = 0;
      c->prof->seen[k] = 0;
    }
  }
  return ARCHE_OK;
}

}  // extern "C"

// ---- equation-of-state averages (Sec. 4): thermalisation cut, mean, error from
// uncorrelated values (integrated autocorrelation time with Sokal's window) ----
extern "C" arche_status arche_eos_average(const double* series, int64_t n, double thermal_fraction,
                                          arche_eos_stat* out) {
  if (!series || !out || n < 0 || !(thermal_fraction >= 0.0 && thermal_fraction < 1.0)) return ARCHE_EINVAL;
  const int64_t start = (int64_t)std::ceil(thermal_fraction * (double)n);
  const int64_t m = n - start;
  if (m < 2) return ARCHE_EINVAL;
  const double* y = series + start;
  for (int64_t i = 0; i < m; ++i)
    if (!std::isfinite(y[i])) return ARCHE_EINVAL;
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i) s += y[i];
  const double mean = s / (double)m;
  double ss = 0.0;
  for (int64_t i = 0; i < m; ++i) ss += (y[i] - mean) * (y[i] - mean);
  const double c0 = ss / (double)m;
  double tau = 0.5;
  if (c0 > 0.0) {
    for (int64_t W = 1; W < m; ++W) {
      double ct = 0.0;
      for (int64_t i = 0; i + W < m; ++i) ct += (y[i] - mean) * (y[i + W] - mean);
      tau += ct / (double)(m - W) / c0;
      if ((double)W >= 5.0 * tau) break;
    }
  }
  const int64_t stride = std::max<int64_t>(1, (int64_t)std::ceil(2.0 * tau));
  const int64_t n_eff = std::max<int64_t>(1, m / stride);
  const double var = ss / (double)(m - 1);
  out->mean = mean;
  out->std = std::sqrt(var);
  out->sem = std::sqrt(var / (double)n_eff);
  out->tau = tau;
  out->n_used = m;
  out->n_eff = n_eff;
  out->stride = stride;
  out->start = start;
  return ARCHE_OK;
}
