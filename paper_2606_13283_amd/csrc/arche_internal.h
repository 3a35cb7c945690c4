// Internal state of one SCF context: device buffers, the device-resident SCF
// scalars, and the kernel launchers shared by the translation units.
#pragma once

#include <atomic>

#include <string>
#include <vector>

#include "../../include/arche.h"
#include "../../include/arche_net.h"
#include "common.h"
#include "fft.h"
#include "profile.h"

// Scalars of the SCF iteration kept on the device (read back by the host only
// to poll convergence).  Written by the kernels of scf.hip.
struct ScfState {
  double mu, N, dN;
  double res;      // ||n_i - n_a|| / ||n_a||
  double K;        // int dn^2 / (dn_a/dmu)
  double Uxc;      // int (v_xc(n_i) - v_xc(n_a)) dn [+ int v_vW[n_i] dn when uvw_w is set]
  double Uvw;      // int (v_vW[n_i] - v_vW[n_a]) dn
  double UH;       // 1/|Omega| sum |dn^|^2 / (pi k^2)
  double w;        // mixing weight of the last iteration
  double maxrel;   // max |dn| / n_a
  double Na;       // int n_a
  int iter;        // completed SCF iterations
  int newton_last;
  int newton_total;
  int done;
  int more_on;
  int mu_fail;
  int err;         // barrier time-out or non-finite value
  int pad;
};

struct GridInfo {
  int N[3];
  int Nh;
  int64_t ng, nh;
  double L[3];
  double vol, dv;
};

// Per-species constants needed inside kernels.
#define ARCHE_MAX_SPECIES 8
struct SpeciesInfo {
  int ns;
  double Z[ARCHE_MAX_SPECIES];
  double rc[ARCHE_MAX_SPECIES];
  // tabulated form factor (null: analytic empty core): non-Coulomb part
  // D_s(q) = V_s(q) + Z_s/(pi q^2) at q = i ff_dq, [ns][ff_len], device
  const double* ff;
  int ff_len;
  double ff_dq;
};

// Device memory of a context: the allocator installed by arche_set_allocator
// when the context was created (null pair: hipMalloc / hipFree).
struct DevAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  hipError_t get(void** p, size_t bytes, hipStream_t s) const {
    if (!alloc) return hipMalloc(p, bytes);
    *p = alloc(bytes, (void*)s);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  void put(void* p, hipStream_t s) const {
    if (!p) return;
    if (release)
      release(p, (void*)s);
    else
      (void)hipFree(p);
  }
};
DevAllocator current_allocator();

// Arguments of the cooperative SCF kernel for one system (scf.hip): steps 1-4
// of an iteration (potential, chemical potential, active density, sums).
struct ActiveArgs {
  const double* Vie;
  const double* VH;
  const double* lap_i;
  const double* n_i;
  double* Vi;
  double* n_a;
  ScfState* st;
  double* part;     // [13][nchunk] chunk partials
  double* res;      // reduced scalars
  unsigned* flags;  // two banks of ARRIVE_LANES arrival counters (grid_allreduce)
  int* err;
  const FdTables* fdt;
  int64_t ng, nchunk;
  double dv, kT, cn, Ne, lam;
  int xc;
  double eta0, tol;
  int mixing, warmup;
  double trust;
  int max_newton;
  int max_iter;  // the iteration that reaches it is the last (done is raised)
  // with More's secant weight and vW: (n_i - n_a)/sqrt(n_a) out, for the pass that
  // sums the v_vW[n_a] part of U_vW, and the v_vW[n_i] part summed with U_xc
  // (null: the U_vW pass does both)
  double* uvw_w;
};

// The rest of an iteration is a fixed sequence of steps; a step that does not
// apply to a system (no von Weizsaecker term, fixed mixing) is left out of its
// list.  The slot says where a step sits in the sequence, so the batched driver
// can run slot s of every system in one launch.
enum {
  SLOT_NHAT_A = 0,     // 3 passes: R2C(n_a) -> n^_a with the U_H partials
  SLOT_LAP_A = 3,      // 3 passes: R2C(sqrt n_a) with the Laplacian (More + vW)
  SLOT_UVW = 6,        // 3 passes: C2R summing U_vW (More + vW)
  SLOT_WEIGHT = 9,     // the mixing weight
  SLOT_HARTREE = 10,   // 3 passes: C2R of n_o^/(pi k^2) forming n_o^ -> V_H
  SLOT_SQRT_O = 13,    // 3 passes: R2C(sqrt n_o) forming n_o, Laplacian (vW)
  SLOT_LAP_O = 16,     // 3 passes: C2R -> lap sqrt(n_o) (vW)
  SLOT_REAL_MIX = 19,  // n_o in real space (no vW)
  SLOT_COUNT = 20
};
enum { STEP_FFT = 0, STEP_WEIGHT = 1, STEP_REAL_MIX = 2 };
struct MixWeightArgs {
  ScfState* st;
  const double* part_h;
  int nbh;
  const double* part_v;
  int nbv;
  int use_vw;
  double vol, dv, w_fixed;
  int bound_drop;  // the weight falls by at most W_MAX_DROP per iteration (the secant form)
  ScfState* ring;  // pinned host ring [ring_n]: the state after iteration t goes to ring[(t - 1) % ring_n] (null: none)
  int ring_n;
};
struct RealMixArgs {
  const ScfState* st;
  double* n_i;
  const double* n_a;
  double* sq;
  int64_t ng;
  int sqrt_when_done;  // 1: once done, sq = sqrt(n_i) (the unfused iteration); 0: nothing
};
struct IterStep {
  int slot, kind;
  unsigned nblocks;
  FftPass fft;
  int dual;     // STEP_FFT: fft and fft2 are independent and launched together
  FftPass fft2;
  MixWeightArgs mw;
  RealMixArgs rm;
};

// SCF iterations per graph launch of a single-context solve, and the host ring
// that holds the states of two launches (the host reads one launch behind)
// words of a context's grid all-reduce counters: two banks (grid_allreduce)
constexpr int SCF_BAR_WORDS = 2 * (int)ARRIVE_BANK;
constexpr int ARCHE_GRAPH_ITERS = 4;
constexpr int ARCHE_RING = 2 * ARCHE_GRAPH_ITERS;

struct arche_ctx {
  arche_params p;  // copy; pointer members are not kept
  std::vector<int32_t> species;
  std::vector<double> Z, rc, mass;
  std::vector<double> ff_host;  // tabulated form factor [ns][ff_len] (empty: analytic)
  double* ff_d = nullptr;
  DevAllocator dalloc_;         // where this context's device memory comes from
  std::vector<double> Zj;  // per atom
  int n_atoms = 0, n_species = 0;
  double Ne = 0, Q = 0, sumZ2 = 0;
  GridInfo g{};
  SpeciesInfo sp{};
  FftPlan plan{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  int coop_blocks = 0;
  std::string err;

  // device fields (real: ng doubles, spectral: nh cplx)
  double *Vie = nullptr, *VH = nullptr, *lap_i = nullptr, *n_i = nullptr, *n_a = nullptr, *Vi = nullptr,
         *lap_a = nullptr, *rtmp = nullptr;
  cplx *nhat_i = nullptr, *nhat_a = nullptr, *ctmp = nullptr, *ctmp2 = nullptr;
  cplx *Sp = nullptr, *Sm = nullptr;  // per species [ns][nh]: S at box k and with Nyquist components negated
  cplx *SZp = nullptr, *SZm = nullptr;
  cplx *prev_nhat = nullptr, *prev_SZp = nullptr, *prev_SZm = nullptr;  // previous converged step
  bool have_prev = false;
  // one-center shells
  int nshell = 0;
  int32_t *shell_of = nullptr, *shell_perm = nullptr, *shell_off = nullptr;
  double *shell_g = nullptr;
  // atoms
  double *pos = nullptr, *Zatom = nullptr, *forces = nullptr, *fpp = nullptr, *fpart = nullptr;
  int32_t *spec_d = nullptr, *sp_order = nullptr, *sp_begin = nullptr;
  cplx *Wp = nullptr, *Wm = nullptr;  // force weights per species [ns][nh]
  cplx *phx = nullptr, *phy = nullptr, *phz = nullptr;  // [n_atoms][N] phase tables
  cplx* phT = nullptr;  // the phase tables transposed, atoms in species order [N_x + N_y + N_h][n_atoms]
  // reductions
  double *partials = nullptr;  // scratch for block partials
  int partial_cap = 0;
  double *sums = nullptr;      // small result vectors
  ScfState *state = nullptr;
  ScfState *state_host = nullptr;  // pinned ring of SCF states, ARCHE_RING entries
  // K whole iterations captured in a HIP graph (fused grids; built at the first solve)
  hipGraph_t iter_graph = nullptr;
  hipGraphExec_t iter_exec = nullptr;
  bool graph_tried = false;
  bool graph_plain = false;  // the captured SCF kernel launch is a plain one
  unsigned *bar = nullptr;         // grid all-reduce arrival counters [scf_bar_words]
  int *err_d = nullptr;
  const FdTables *fdt = nullptr;

  // host copies of the last solve
  std::vector<double> h_pos, h_forces;
  bool solved = false, converged = false, forces_ready = false;
  double eta0 = 0;  // I_{1/2}^{-1}(n0/c_n)
  arche_result last{};
  // MD state
  std::vector<double> r_prev;
  bool have_r_prev = false;
  // optional per-kernel timing
  Profiler* prof = nullptr;
  // launch arguments of an iteration (fixed for the life of the context)
  bool iter_built = false, fused = false;
  ActiveArgs active{};
  std::vector<IterStep> steps;
  arche_net* init_net = nullptr;  // learned initial density (not owned)
  std::vector<ScfState> hist;     // polled SCF states of the last single solve
};

// host Fermi-Dirac integrals: j = 0, 1, 2 for I_{-1/2}, I_{1/2}, I_{3/2}; the inverse of I_{1/2}
double host_fd(int j, double x);
double host_fd_inverse_p12(double y);

// device Fermi-Dirac tables (uploaded once per process and device)
const FdTables* fd_tables_device(int device);

// kernels_*.hip launchers ---------------------------------------------------
// reductions
int red_blocks(int64_t n);
hipError_t finish_sums(const double* partials, int nblk, int nsum, double* out, hipStream_t s);

// SCF (scf.hip)
hipError_t scf_iteration(arche_ctx* c);
bool scf_plain_launch(const arche_ctx* c);  // the SCF kernel's next launch is a plain one
// contexts alive in the process (arche_scf_init .. arche_scf_free, batch members included)
extern std::atomic<int> g_live_contexts;
hipError_t scf_reset_state(arche_ctx* c, double mu0);
hipError_t scf_vw_laplacian(arche_ctx* c, const double* n, double* lap);  // lap = del^2 sqrt(n)
hipError_t scf_sqrt_spectrum(arche_ctx* c, const double* n, cplx* out);   // out = (|Omega|/N_g) DFT(sqrt n)
hipError_t scf_energies(arche_ctx* c, double* out16);  // see scf.hip for the order
hipError_t scf_initial_uniform(arche_ctx* c);
hipError_t scf_initial_one_center(arche_ctx* c, int* used_fallback);  // ionic.hip
// n_i only; raw: unfloored copy; delta: the superposition's change since the
// previous step (ionic.hip)
hipError_t scf_one_center_density(arche_ctx* c, int* used_fallback, double* raw, double* delta);
hipError_t scf_floor_renorm(arche_ctx* c, double* n, bool* ok);       // ionic.hip
hipError_t scf_add_scalar(arche_ctx* c, double* x, double v);         // x += v (ionic.hip)
hipError_t scf_learned_proposal(arche_ctx* c);  // rtmp: network output r -> proposal (ionic.hip)
hipError_t scf_prepare_input(arche_ctx* c);  // n^_i, V_H, lap sqrt(n_i) from n_i
int scf_coop_blocks(int64_t ng);
// the iteration's launch arguments (fills c->active, c->steps, c->fused)
void scf_build_iteration(arche_ctx* c);
hipError_t scf_step_launch(const IterStep& st, hipStream_t s);
// batched forms (one launch for many systems)
int scf_batch_capacity();  // co-resident blocks of the batched cooperative kernel
hipError_t scf_active_batch_launch(const ActiveArgs* args, const int* group_begin, int nsys, int nblocks,
                                   hipStream_t s);
hipError_t scf_weight_batch_launch(const MixWeightArgs* jobs, int njobs, hipStream_t s);
hipError_t scf_real_mix_batch_launch(const RealMixArgs* jobs, const int* bbeg, int njobs, unsigned nblocks,
                                     hipStream_t s);
unsigned scf_real_mix_blocks(int64_t ng);
size_t scf_part_offset(const arche_ctx* c);  // start of the non-cooperative partials

// ionic (ionic.hip)
hipError_t ionic_structure(arche_ctx* c);  // phases, S+/S-, SZ, V^ie
hipError_t ionic_forces(arche_ctx* c, const cplx* nhat, double* forces_dev);
hipError_t ionic_ewald(arche_ctx* c, double* U3 /*host: pp, pm, je*/, double alpha);
hipError_t ionic_pressure_ie(arche_ctx* c, const cplx* nhat, double* out /*host*/);
hipError_t ionic_shells(arche_ctx* c);
hipError_t ionic_stress_sums(arche_ctx* c, const cplx* nhat, const cplx* shat, double alpha, double* out24,
                             double* pp6);
size_t ionic_force_partials(const arche_ctx* c);
double ewald_alpha(const arche_ctx* c);

// runtime.hip: the phases of one solve, shared with the batched driver
arche_status solve_begin(arche_ctx* c, const double* pos_host, int init, int* fallback);  // ionic field, guess, reset
arche_status solve_collect(arche_ctx* c, arche_result* out);  // SCF state -> out
arche_status solve_finish(arche_ctx* c, arche_result* out, int fallback);  // energies, pressure, history
arche_status solve_forces(arche_ctx* c);  // forces -> c->h_forces
arche_status ctx_error(arche_ctx* c, arche_status s, const std::string& m);
