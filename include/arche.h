/*
 * arche.h -- C ABI of the MI355X (gfx950) FP64 orbital-free SCF library
 * (libarche.so).  The method is the one of "Arche, an orbital-free molecular
 * dynamics code for fast production of equations of state": a finite-temperature
 * Thomas-Fermi (+ lambda von Weizsaecker, + LDA exchange-correlation) electron
 * density on a periodic grid, found by a self-consistent-field (SCF) iteration
 * with a Newton search of the chemical potential and More's optimal mixing,
 * followed by free energy, pressure and ionic forces, inside a Verlet MD loop.
 *
 * Conventions for every call:
 *   - Hartree atomic units, FP64, C row-major arrays.
 *   - Real grid fields are [Nx][Ny][Nz] (z fastest); grid point
 *     (i,j,k) sits at (i Lx/Nx, j Ly/Ny, k Lz/Nz) (Sec. 2.3).
 *   - Pointers named *_host are host memory owned by the caller; the library
 *     copies in/out and keeps no reference after the call returns.
 *   - The context owns all device memory it allocates (on the device current
 *     at arche_scf_init, through the allocator installed by arche_set_allocator
 *     at that time, else hipMalloc) and frees it in arche_scf_free.
 *   - Every call returns an arche_status; no call aborts or prints.  After an
 *     error, arche_last_error(ctx) describes it.
 *   - A context is used by one host thread at a time.
 */
#ifndef ARCHE_H
#define ARCHE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arche_ctx arche_ctx;

typedef enum {
  ARCHE_OK = 0,
  ARCHE_EINVAL = -1,  /* invalid argument (sizes, NaN/inf positions, bad grid) */
  ARCHE_ENOMEM = -2,  /* device or host allocation failed */
  ARCHE_EHIP = -3,    /* a HIP runtime call failed */
  ARCHE_ENOCONV = -4, /* SCF (or the mu search) did not converge; results hold the last iterate */
  ARCHE_ESTATE = -5   /* call not valid in the current state (e.g. forces before a solve) */
} arche_status;

/* initial density of an SCF solve (Sec. 2.5, 2.5.1) */
enum {
  ARCHE_INIT_UNIFORM = 0,    /* n_0 = N_e / |Omega| */
  ARCHE_INIT_ONE_CENTER = 1, /* superposition guess from the previous converged step; uniform if none */
  ARCHE_INIT_KEEP = 2,       /* the context's current density (e.g. from arche_set_density) */
  ARCHE_INIT_LEARNED = 3     /* the learned proposal of arche_net.h; one-center if none */
};
/* density mixing (Sec. 2.5.2) */
enum {
  ARCHE_MIX_FIXED = 0,       /* n_o = n_a + w_fixed (n_i - n_a) throughout */
  ARCHE_MIX_MORE = 1,        /* More's weight w = U/(U+K) with U over every potential term (Hartree, xc, vW)
                                as the secant int (V_i - V_eff[n_a]) dn and K the secant int kT (eta(n_i) - eta_a) dn,
                                its fall bounded by 0.05 per iteration */
  ARCHE_MIX_MORE_PRINTED = 2 /* More's weight exactly as printed: U = int int dn dn'/|r-r'| (Hartree only),
                                K = int dn^2/(dn_a/dmu), no bound on its fall */
};
/* exchange-correlation */
enum { ARCHE_XC_NONE = 0, ARCHE_XC_LDA = 1 /* Dirac exchange + Perdew-Zunger 1981 correlation */ };

typedef struct {
  int32_t n_atoms;          /* N_i >= 1 */
  int32_t n_species;        /* 1..8 */
  const int32_t *species;   /* [n_atoms], values in [0, n_species) */
  const double *Z;          /* [n_species] ionic charge Z_s > 0 */
  const double *rc;         /* [n_species] empty-core radius r_c >= 0 (bohr): form factor
                               V_s(k) = -Z_s cos(2 pi |k| r_c) / (pi |k|^2), k in 1/bohr (Sec. 2.4) */
  const double *mass;       /* [n_species] ionic mass, electron masses (MD only) */
  double cell[3];           /* orthorhombic cell edges L_x, L_y, L_z (bohr) */
  int32_t grid[3];          /* N_x, N_y, N_z: even, factors 2, 3, 5 only, <= 1024 */
  double kT;                /* electron temperature k_B T_e (Hartree) > 0 */
  double lambda_vw;         /* von Weizsaecker coefficient lambda >= 0 */
  int32_t xc;               /* ARCHE_XC_* */
  double scf_tol;           /* stop when ||n_i - n_a||_2 / ||n_a||_2 < scf_tol */
  int32_t scf_max_iter;     /* > 0 */
  int32_t mixing;           /* ARCHE_MIX_* */
  int32_t more_warmup;      /* More weight allowed from this iteration on (e.g. 3) */
  double more_trust;        /* ... once max |n_i - n_a| / n_a <= more_trust (e.g. 0.5) */
  double w_fixed;           /* fixed weight w of n_o = n_a + w (n_i - n_a) (e.g. 0.95) */
  int32_t init;             /* ARCHE_INIT_* for arche_scf_solve */
  /* Optional fields below: zero (e.g. a zero-initialised struct) selects the default. */
  const double *ff_table;   /* NULL: the analytic empty-core form factor of rc.  Otherwise a
                               tabulated local pseudopotential (eq. iepseudo takes any radial
                               V_s(|k|)), [n_species][ff_len] samples of its non-Coulomb part
                               D_s(q) = V_s(q) + Z_s / (pi q^2) at q = i * ff_dq (q = |k| in
                               1/bohr, i = 0..ff_len-1).  D_s(0), the limit q -> 0, is the
                               k = 0 term of E^ie (Sec. 2.6.5).  Between nodes D_s is the cubic
                               through the nodes i-1, i, i+1, i+2 around q (local cubic
                               Lagrange, with D_s(-q) = D_s(q) at the first interval), and
                               dV_s/dq, which enters the pressure, is that cubic's derivative
                               plus 2 Z_s / (pi q^3).  The table must extend two nodes past
                               the largest |k| of the grid (EINVAL otherwise).  rc is then
                               not used.  Copied at init. */
  int32_t ff_len;           /* nodes per species (>= 4 when ff_table is set) */
  double ff_dq;             /* node spacing in 1/bohr (> 0 when ff_table is set) */
  double ewald_alpha;       /* Ewald splitting parameter (1/bohr) of Sec. 2.6.3; <= 0: the
                               automatic sqrt(pi k_c / r_c), k_c = min N/(2L), r_c = min L/2 */
  int32_t exclusive_device; /* nonzero: the caller guarantees that nothing else runs on the
                               device during this context's solves (no other process, no
                               other live arche context); the SCF kernel, whose grid-wide
                               reductions need all its blocks resident, is then a plain launch
                               (~20 us less per iteration than a cooperative one).  0: a
                               cooperative launch, which guarantees residency. */
} arche_params;

/* Energy terms (Hartree), index into arche_result.terms */
enum {
  ARCHE_T_FTF = 0,  /* int f0(n): Thomas-Fermi free energy */
  ARCHE_T_KE,       /* K_e = (3/2) int p0: TF kinetic energy (Sec. 2.6.2) */
  ARCHE_T_FVW,      /* von Weizsaecker energy */
  ARCHE_T_EH,       /* Hartree energy U^ee (Sec. 2.6.4) */
  ARCHE_T_FXC,      /* xc energy */
  ARCHE_T_EIE,      /* electron-ion energy E^ie incl. the k=0 non-Coulomb term (Sec. 2.6.5) */
  ARCHE_T_UII,      /* Ewald ion-ion energy U^ii (Sec. 2.6.3) */
  ARCHE_T_UPP,
  ARCHE_T_UPM,
  ARCHE_T_UJE,
  ARCHE_T_ALPHA,    /* Ewald splitting parameter used */
  ARCHE_T_COUNT
};
/* Pressure terms (Hartree/bohr^3), index into arche_result.pterms */
enum { ARCHE_P_TF = 0, ARCHE_P_VW, ARCHE_P_H, ARCHE_P_XC, ARCHE_P_IE, ARCHE_P_II, ARCHE_P_COUNT };

typedef struct {
  double F;                       /* free energy F = F_TF + F_vW + E_H + F_xc + E^ie + U^ii */
  double E;                       /* internal energy (K_e in place of F_TF) */
  double terms[ARCHE_T_COUNT];
  double P;                       /* pressure without the ionic kinetic term */
  double pterms[ARCHE_P_COUNT];
  double mu;                      /* chemical potential */
  double residual;                /* final ||n_i - n_a|| / ||n_a|| */
  double w_last;                  /* last mixing weight */
  int32_t scf_iters;
  int32_t newton_iters;           /* total Newton passes of the mu search */
  int32_t used_fallback;          /* the requested guess was replaced (one-center by uniform, learned by one-center) */
  int32_t converged;
} arche_result;

/* Create a context for one system (Sec. 2.3 grid, Sec. 2.4 pseudopotential).
 * p: problem statement, copied (its arrays are copied too).
 * hip_stream: hipStream_t to run on, or NULL for a stream the context creates.
 * out: receives the context.  EINVAL on invalid parameters, ENOMEM/EHIP on
 * device failures (no context is returned then). */
arche_status arche_scf_init(const arche_params *p, void *hip_stream, arche_ctx **out);

/* Solve the SCF (Sec. 2.5) for ions at pos_host [n_atoms][3] (bohr; wrapped
 * into the cell), then evaluate free energy and pressure (Sec. 2.6) into *out.
 * The initial density follows p.init.  ENOCONV if the SCF did not reach
 * scf_tol within scf_max_iter (out still describes the last iterate), EINVAL
 * for non-finite positions. */
arche_status arche_scf_solve(arche_ctx *ctx, const double *pos_host, arche_result *out);

/* Ionic forces F_j = F^ie + F^pm + F^pp (eq. force; Sec. 2.6.3, 2.6.5) at the
 * last converged solve, into forces_host [n_atoms][3] (Hartree/bohr).
 * ESTATE if there is no converged solve. */
arche_status arche_forces(arche_ctx *ctx, double *forces_host);

/* One Verlet step (Sec. 2.1).  On entry pos_io holds r(t) and vel_io v(t); if
 * the context has no converged solve at r(t) one is made first.  The step sets
 * r(t+dt) = 2 r(t) - r(t-dt) + F(t)/m dt^2 (with r(t-dt) = r(t) - v dt +
 * F dt^2/(2m) on the first step), solves the SCF at r(t+dt) (initial density
 * per p.init, normally one-center) and returns r(t+dt) in pos_io, the central
 * difference v(t) = (r(t+dt) - r(t-dt)) / (2 dt) in vel_io, F(t+dt) in
 * forces_out_host [n_atoms][3] (may be NULL) and the solve's result in *out.
 * Positions are not wrapped on output. */
arche_status arche_md_step(arche_ctx *ctx, double dt, double *pos_io, double *vel_io,
                           double *forces_out_host, arche_result *out);

/* Stress tensor terms (Sec. 2.6), index of the 3x3 blocks of arche_stress's terms */
enum {
  ARCHE_S_KIN = 0, /* sigma^i = -(1/|Omega|) sum_j m_j v_mu v_nu (Sec. 2.6.1; zero without velocities) */
  ARCHE_S_TF,      /* sigma^e of the Thomas-Fermi term, -(1/|Omega|) int p0 delta (Sec. 2.6.2) */
  ARCHE_S_VW,      /* von Weizsaecker: -(lambda (2 pi)^2/|Omega|^2) sum_k k_mu k_nu |s^(k)|^2, s = sqrt(n) */
  ARCHE_S_XC,      /* LDA xc: -(1/|Omega|) int n (v_xc - eps_xc) delta */
  ARCHE_S_EE,      /* Hartree sigma^ee (Sec. 2.6.4) */
  ARCHE_S_IE,      /* electron-ion sigma^ie (Sec. 2.6.5) */
  ARCHE_S_II,      /* Ewald sigma^pp + sigma^pm + sigma^je at the context's alpha held fixed (Sec. 2.6.3) */
  ARCHE_S_COUNT
};

/* Stress tensor Sigma = sum of the terms above at the last converged solve,
 * each (1/|Omega|) times the derivative of its energy under a homogeneous
 * strain at fixed fractional positions (so P = -tr(Sigma)/3 without the
 * kinetic term reproduces arche_result.P, the Ewald part to the Ewald
 * truncation since arche_result takes U^ii as independent of alpha).
 * vel_host [n_atoms][3] (may be NULL: no kinetic term); sigma_host [3][3]
 * receives the total (Hartree/bohr^3); terms_host (may be NULL)
 * [ARCHE_S_COUNT][3][3] the terms.  ESTATE without a converged solve. */
arche_status arche_stress(arche_ctx *ctx, const double *vel_host, double *sigma_host, double *terms_host);

/* The positions r(t+dt) that arche_md_step would move to from pos_host with
 * vel_host (the Verlet update of Sec. 2.1 with the forces of the converged
 * solve at pos_host and the context's r(t-dt), or the Taylor start when it has
 * none), into next_host [n_atoms][3]; nothing is solved and the context's
 * state is unchanged.  ESTATE without a converged solve at exactly pos_host. */
arche_status arche_md_predict(arche_ctx *ctx, double dt, const double *pos_host, const double *vel_host,
                              double *next_host);

/* Copy the converged density n_a [Nx][Ny][Nz] to dst (host if
 * dst_on_device == 0, else device memory on the context's device).  ESTATE
 * before a solve. */
arche_status arche_get_density(arche_ctx *ctx, double *dst, int32_t dst_on_device);

/* Replace the context's input density (used by the next solve with
 * p.init == ARCHE_INIT_KEEP); src [Nx][Ny][Nz] host or device as above.  The
 * density must be positive; it is rescaled to N_e electrons. */
arche_status arche_set_density(arche_ctx *ctx, const double *src, int32_t src_on_device);

/* Forget the previous step (next one-center guess falls back to uniform). */
arche_status arche_reset_history(arche_ctx *ctx);

void arche_scf_free(arche_ctx *ctx);

/* Device memory of contexts and batches created from now on (Sec. 5.2 keeps
 * every field resident on the GPU for the whole run; this lets the caller's
 * memory manager, e.g. PyTorch's caching allocator, supply it).
 * alloc(bytes, stream) returns device memory on the current device, aligned
 * to 256 bytes, or NULL on failure (the init call then returns ENOMEM);
 * release(ptr, stream) gives it back.  `stream` is the context's hipStream_t.
 * A context keeps the pair it was created with and releases through it in
 * arche_scf_free, whatever is installed by then.  Both NULL: hipMalloc /
 * hipFree again.  EINVAL if exactly one is NULL.  Process-wide; not
 * synchronised with concurrent arche_scf_init calls on other threads. */
arche_status arche_set_allocator(void *(*alloc)(size_t bytes, void *stream),
                                 void (*release)(void *ptr, void *stream));

/* Per-context message of the last error (empty if none); valid until the next
 * call on ctx.  With ctx == NULL, the message of the last failed arche_scf_init
 * in this thread. */
const char *arche_last_error(const arche_ctx *ctx);

const char *arche_version(void);

/* ---- Average-atom pseudopotential (Sec. 2.4) -------------------------------
 * A finite-temperature Thomas-Fermi (+ LDA when xc = ARCHE_XC_LDA) average atom:
 * a nucleus of charge Z in its Wigner-Seitz sphere (4/3 pi r_ws^3 rho_ion = 1),
 * neutral inside it, solved self-consistently on a radial grid (n_radial nodes
 * uniform in ln r from 1e-7 r_ws to r_ws, trapezoid rule in ln r).  Inside
 * r_cut (the first node at or beyond r_cut_frac r_ws) its density is replaced
 * by exp(a + b r^2 + c r^4) with the same value, slope and charge at r_cut; the
 * pseudopotential is the potential whose TF + Hartree + xc response is that
 * pseudo-density, V~ = mu - kT I_{1/2}^{-1}(n~/c_n) - v_xc(n~) - V_H[n~] inside
 * r_cut and -Z/r outside.  table_out[k], k < n_q, receives its non-Coulomb
 * form factor D(k dq) = 4 pi int (V~ + Z/r) r^2 sin(2 pi q r)/(2 pi q r) dr,
 * in the form arche_params.ff_table takes (for one species; ff_dq = dq).
 * out->dE_AA is Delta E_AA, the internal energy of the average atom with the
 * Coulomb potential minus that with the pseudopotential (Hartree per atom; the
 * paper adds it to the internal energy per ion).  Host-only.  EINVAL for bad
 * parameters, ENOCONV if the average atom does not converge. */
typedef struct {
  double Z;          /* nuclear charge (every electron of the atom) */
  double rho_ion;    /* ion number density (1/bohr^3) */
  double kT;         /* electron temperature (Hartree) */
  double r_cut_frac; /* r_cut / r_ws in (0, 1) */
  int32_t xc;        /* ARCHE_XC_NONE or ARCHE_XC_LDA */
  int32_t n_radial;  /* radial nodes (>= 101; e.g. 2001) */
} arche_aa_params;
typedef struct {
  double r_ws, r_cut, mu, dE_AA, a, b, c;
  int32_t iters;
} arche_aa_result;
arche_status arche_aa_pseudopotential(const arche_aa_params *p, double dq, int32_t n_q, double *table_out,
                                      arche_aa_result *out);

/* ---- Equation-of-state averages (Sec. 4, Fig. pressurehistory) -----------
 * The time average of an MD observable (pressure, energy) after dropping the
 * thermalisation part, with the error from uncorrelated values.  Host-only.
 * Kept values x_t, t = start .. n-1 with start = ceil(thermal_fraction n)
 * (the paper drops about 20 %).  tau = 1/2 + sum_{t=1}^{W} C(t)/C(0),
 * C(t) = (1/(m-t)) sum_i (x_i - mean)(x_{i+t} - mean), summed to the first
 * window W >= 5 tau (Sokal's automatic window); values 2 tau apart count as
 * uncorrelated: stride = max(1, ceil(2 tau)), n_eff = max(1, m / stride),
 * sem = sqrt(var / n_eff) with var the unbiased sample variance.  EINVAL if
 * fewer than two values remain, a kept value is not finite, or
 * thermal_fraction is outside [0, 1). */
typedef struct {
  double mean, std, sem, tau;
  int64_t n_used, n_eff, stride, start;
} arche_eos_stat;
arche_status arche_eos_average(const double *series, int64_t n, double thermal_fraction, arche_eos_stat *out);

/* ---- Batched solves: many independent snapshots on one GPU ----------------
 * A batch holds one context per snapshot (each its own cell, grid, atoms,
 * temperature and SCF options) on one stream.  arche_batch_solve runs the SCF
 * of every snapshot together: each pass of an iteration is ONE launch over all
 * unconverged snapshots of any grid size, the iterations are captured in a HIP
 * graph, and a snapshot drops out when its own convergence test passes.  Per
 * snapshot the arithmetic is exactly that of arche_scf_solve on the same
 * context, so results are bit-identical to unbatched solves.  Scheduling
 * choices (blocks per snapshot in the cooperative kernel, iterations per graph
 * launch) are made by an autotuner on the first solve; none of them changes a
 * result bit.  Supported: grids whose three edges are in {16, 20, 24, 30, 32,
 * 40, 48, 50, 54, 60, 64, 72, 80, 96}. */
typedef struct arche_batch arche_batch;

/* p: n_snap problem statements (copied).  hip_stream as in arche_scf_init.
 * EINVAL for invalid parameters or a grid outside the batched set. */
arche_status arche_batch_init(int32_t n_snap, const arche_params *p, void *hip_stream, arche_batch **out);

/* pos_host[i]: positions [n_atoms_i][3] of snapshot i.  out[i] receives its
 * result; forces_host (may be NULL) gives per snapshot a caller array
 * [n_atoms_i][3] for the forces, or NULL entries to skip.  Returns ENOCONV if
 * any snapshot did not converge (see out[i].converged), else OK. */
arche_status arche_batch_solve(arche_batch *b, const double *const *pos_host, arche_result *out,
                               double *const *forces_host);

/* The context of snapshot i (owned by the batch): density, debug and single
 * solves on it behave as for a context from arche_scf_init. */
arche_ctx *arche_batch_context(arche_batch *b, int32_t i);

/* Scheduling of the last solve: info[0] = cooperative blocks of the first
 * iteration, info[1] = iterations per graph launch, info[2] = 1 if whole
 * iterations (cooperative kernel included) were graph-captured, 0 if only the
 * passes after it, info[3] = graph launches, info[4] = times the active set was
 * compacted, info[5] = 1 if the autotuner measured (0: cached or forced). */
arche_status arche_batch_info(const arche_batch *b, int32_t info[6]);

/* Force the schedule (0 = let the autotuner choose): blocks of the cooperative
 * kernel and iterations per graph launch.  For tests of result independence. */
arche_status arche_batch_set_schedule(arche_batch *b, int32_t coop_blocks, int32_t iters_per_graph);

const char *arche_batch_last_error(const arche_batch *b);
void arche_batch_free(arche_batch *b);

/* One-shot form: init, solve, free. */
arche_status arche_scf_solve_batch(int32_t n_snap, const arche_params *p, const double *const *pos_host,
                                   arche_result *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ARCHE_H */
