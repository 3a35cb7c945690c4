// SCF iteration kernels (paper Sec. 2.5): potential assembly, Newton search of
// mu, active density, More mixing weight, mixed density, Hartree and von
// Weizsaecker potentials; and the energy reductions of Sec. 2.6.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "arche_internal.h"
#include "profile.h"

namespace {

constexpr double PI = 3.14159265358979323846;


// The SCF kernel runs blocks of SCF_THREADS threads.  The grid is cut into
// nchunk chunks of SCF_CHUNK points: the grid is read as PPT stripes of
// nchunk*SCF_THREADS points, and chunk c takes the c-th run of SCF_THREADS
// consecutive points in each stripe (thread t the t-th of each).  A
// chunk thus samples the whole cell, and blocks near ions and between them carry
// the same mix of work; each wave still reads 64 consecutive values.  Every
// global sum is a sum of per-chunk partials in chunk order, so the result does
// not depend on how many blocks share the work (a batched solve, with fewer
// blocks per snapshot, is bit-identical to an unbatched one).  The kernel's
// FP64 evaluations need about 200 registers per lane, so two waves per SIMD
// (two blocks per CU, whose LDS caches then fill the CU) is what fits without
// spilling.
constexpr int SCF_THREADS = 256;
constexpr int PPT = 16;
// More's weight may switch on once mu moves by at most this fraction of kT
// between iterations (the chemical-potential fluctuations of Sec. 2.5.2 are small)
constexpr double MU_SETTLED = 0.02;
// More's weight may fall by at most this much from one iteration to the next
// (the quadratic model can send it to 0 in one step in low-density regions)
constexpr double W_MAX_DROP = 0.05;
constexpr int SCF_CHUNK = SCF_THREADS * PPT;
// the chemical potential is found once |N(mu) - N_e| <= MU_TOL N_e
constexpr double MU_TOL = 1e-14;
// after a Newton evaluation with |N - N_e| <= SPEC_NEWTON N_e the next pass is
// most likely the last (quadratic convergence) and forms the active sums too
constexpr double SPEC_NEWTON = 1e-7;
// LDS doubles for block_reduce_n<8>
constexpr int RED_SH = (SCF_THREADS / 64) * 8;

// point q of this thread in chunk c (>= ng: none)
__device__ inline int64_t chunk_point(const ActiveArgs& a, int64_t c, int q) {
  return (int64_t)q * (a.nchunk * SCF_THREADS) + c * SCF_THREADS + threadIdx.x;
}

// The first NV block-reduced values of acc go to slots s0.. of chunk c.
template <int NV>
__device__ inline void put_chunk_n(const double* acc, double* part, int s0, int64_t nchunk, int64_t c) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) coherent_store(part + (int64_t)(s0 + k) * nchunk + c, acc[k]);  // read by grid_allreduce
  }
}

// Points are processed in groups of PG: the group's loads are issued together
// (at indices clamped into the grid, so a ragged tail needs no branch), the
// common paths (the interval polynomial of I_{1/2}, the r_s >= 1 branch of the
// LDA, the cubic K shift) run branch-free so the points' evaluations interleave,
// and the rare cases are redone for the lanes that need them.
constexpr int PG = 2;

// I_{1/2} and D derivatives at x[g] for a group
template <int D>
__device__ inline void fd_group(const FdLds& fdl, const double* x, double (*d)[D + 1]) {
#pragma unroll
  for (int g = 0; g < PG; ++g) fd_p12_poly<D>(fdl, x[g], d[g]);
  bool out = false;
#pragma unroll
  for (int g = 0; g < PG; ++g) out |= !fd_p12_in_poly(x[g]);
  if (out) {
#pragma unroll
    for (int g = 0; g < PG; ++g)
      if (!fd_p12_in_poly(x[g])) fd_p12_derivs<D>(fdl, x[g], d[g]);
  }
}

// v_xc(n[g]) for a group
__device__ inline void vxc_group(const double* n, double* v) {
  bool hi[PG], any = false;
#pragma unroll
  for (int g = 0; g < PG; ++g) {
    v[g] = lda_vxc_low(n[g], hi[g]);
    any |= hi[g];
  }
  if (any) {
#pragma unroll
    for (int g = 0; g < PG; ++g)
      if (hi[g]) lda_xc(n[g], v[g]);
  }
}

// Sums for one chunk at chemical potential mu, eta = (mu - V_i)/kT:
//   slots 0, 1: sum I_{1/2}(eta), sum dI_{1/2}/deta (N(mu) and N'(mu) up to
//               the factors dv c_n and dv c_n / kT)
// and with ACTIVE, which also stores n_a = c_n I_{1/2}(eta):
//   slots 2..7: sum dn^2, sum n_a^2, K, U_xc, sum n_a, max |dn|/n_a
//   (dn = n_i - n_a; K is the secant of the Thomas-Fermi potential kT eta(n)
//   between n_a and n_i, U_xc the same for v_xc; both only with with_k, else 0:
//   the secant K inverts I_{1/2} at n_i, costly while n_i and n_a are far apart,
//   and only More's weight uses it)
// Two blocks share each CU, and a SIMD issues from the older block's waves
// first when both are ready, so the younger one used to end a phase ~5 us after
// the older one while the grid-wide reduction waited for it.  The first and the
// second half of the grid (dispatched in that order, one block per CU each)
// take turns at the higher wave priority from one group of points to the next,
// so that both blocks of a CU finish a phase together.  Scheduling only: the
// arithmetic and its order are unchanged.
__device__ inline void take_turn(int group, bool young) {
  if (((group & 1) != 0) == young) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// With CACHE, vls and xls (LDS, [PPT][SCF_THREADS]) hold the block's V_i and
// v_xc(n_i) from the assembly.
// FULL: every point of the chunk lies in the grid (N_g a multiple of SCF_CHUNK),
// so the ragged-tail selects fold away.
template <bool CACHE, bool ACTIVE, bool FULL = false>
__device__ inline void chunk_sums(const ActiveArgs& a, int64_t c, const double* vls, const double* xls, double mu,
                                  double ikT, const FdLds& fdl, double* sh, bool with_k = true, bool young = false) {
  const bool more = a.mixing == ARCHE_MIX_MORE && with_k;  // secant K and U_xc
  const bool printed = a.mixing == ARCHE_MIX_MORE_PRINTED;  // K = int dn^2 / (dn_a/dmu)
  const double icn = 1.0 / a.cn;
  constexpr int D = ACTIVE ? 3 : 1;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int q0 = 0; q0 < PPT; q0 += PG) {
    take_turn(q0 / PG, young);
    int64_t ip[PG];
    bool ok[PG];
    double x[PG], ni[PG];
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      const int64_t i = chunk_point(a, c, q0 + g);
      ok[g] = FULL || i < a.ng;
      ip[g] = ok[g] ? i : a.ng - 1;
      const double v = CACHE ? vls[(q0 + g) * SCF_THREADS + threadIdx.x] : a.Vi[ip[g]];
      x[g] = (mu - v) * ikT;
      if (ACTIVE) ni[g] = a.n_i[ip[g]];
    }
    double d[PG][D + 1];
    fd_group<D>(fdl, x, d);
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      acc[0] += ok[g] ? d[g][0] : 0.0;
      acc[1] += ok[g] ? d[g][1] : 0.0;
    }
    if (ACTIVE) {
      double na[PG], dn[PG];
#pragma unroll
      for (int g = 0; g < PG; ++g) {
        na[g] = a.cn * d[g][0];
        dn[g] = ni[g] - na[g];
        if (ok[g]) a.n_a[ip[g]] = na[g];
        acc[2] += ok[g] ? dn[g] * dn[g] : 0.0;
        acc[3] += ok[g] ? na[g] * na[g] : 0.0;
      }
      if (more) {
        double sh_[PG];
        bool far[PG], anyfar = false;
#pragma unroll
        for (int g = 0; g < PG; ++g) {
          sh_[g] = fd_p12_shift_cubic(ni[g] * icn, d[g], far[g]);
          anyfar |= far[g] && ok[g];
        }
        if (anyfar) {
          // moderate shifts by the cubic model polished with one Newton step,
          // larger ones by the full inversion
          bool farther[PG], anyfarther = false;
#pragma unroll
          for (int g = 0; g < PG; ++g) {
            farther[g] = far[g] && ok[g] && !fd_p12_shift_near(fdl, ni[g] * icn, x[g], d[g], sh_[g]);
            anyfarther |= farther[g];
          }
          if (anyfarther) {
#pragma unroll
            for (int g = 0; g < PG; ++g)
              if (farther[g]) sh_[g] = fd_p12_inverse_from(fdl, ni[g] * icn, x[g], d[g][0], d[g][1]) - x[g];
          }
        }
#pragma unroll
        for (int g = 0; g < PG; ++g) acc[4] += ok[g] ? a.kT * sh_[g] * dn[g] : 0.0;  // kT (eta_i - eta_a) dn
        if (a.uvw_w) {
          // U_vW's v_vW[n_i] part, v_vW[n] = -(lambda/2) lap(sqrt n)/sqrt n, with U_xc;
          // dn/sqrt(n_a) for the pass that sums the v_vW[n_a] part
#pragma unroll
          for (int g = 0; g < PG; ++g) {
            const double li = a.lap_i[ip[g]];
            acc[5] += ok[g] ? -0.5 * a.lam * li * rsqrt_nr(ni[g]) * dn[g] : 0.0;
            if (ok[g]) a.uvw_w[ip[g]] = dn[g] * rsqrt_nr(na[g]);
          }
        }
      }
      if (printed) {
        // dn_a/dmu = (c_n / kT) dI_{1/2}/deta
#pragma unroll
        for (int g = 0; g < PG; ++g) acc[4] += ok[g] ? dn[g] * dn[g] * a.kT / (a.cn * d[g][1]) : 0.0;
      }
      if (a.xc && more) {
        double va[PG], vi[PG];
        vxc_group(na, va);
        if (CACHE) {
#pragma unroll
          for (int g = 0; g < PG; ++g) vi[g] = xls[(q0 + g) * SCF_THREADS + threadIdx.x];
        } else {
          vxc_group(ni, vi);
        }
#pragma unroll
        for (int g = 0; g < PG; ++g) acc[5] += ok[g] ? (vi[g] - va[g]) * dn[g] : 0.0;
      }
#pragma unroll
      for (int g = 0; g < PG; ++g) {
        acc[6] += ok[g] ? na[g] : 0.0;
        acc[7] = ok[g] ? fmax(acc[7], fabs(dn[g]) / na[g]) : acc[7];
      }
    }
  }
  __builtin_amdgcn_s_setprio(0);
  block_reduce_n<ACTIVE ? 8 : 2>(acc, ACTIVE ? 0x80u : 0u, sh);
  put_chunk_n<ACTIVE ? 8 : 2>(acc, a.part, 0, a.nchunk, c);
}

// Steps 1-4 of one SCF iteration for one system, run by a group of G
// co-resident blocks (lb = this block's index in the group).
//   1. V_i = V^ie + V_H + v_xc(n_i) + v_vW[n_i] with its sum, max and min, and
//      at the previous iteration's mu the sums of I_{1/2} and of its first
//      three derivatives: N(mu) and the cubic Taylor model of ln N about that mu
//   2. Newton search of mu (safeguarded by bisection) for ln N(mu) = ln N_e,
//      started from the root of the cubic model: mu moves little between
//      iterations, so the model's root is usually exact to MU_TOL and one pass
//      confirms it; in the first iterations, where mu moves by several kT,
//      ln N (nearly linear in mu where N grows exponentially) keeps the steps
//      few where Newton on N itself would advance about kT per pass
//   3. n_a at mu with the sums of the residual and of More's weight; a Newton
//      pass that is expected to be the last forms them too, so when it
//      converges no separate pass is needed
//   4. the SCF scalars (block 0)
// grid_allreduce hands every block of the group the same fixed-order result, so
// all of them take the same branches.  With CACHE (at most one chunk per block)
// V_i and v_xc(n_i) stay in LDS between the phases; V_i is stored only by the
// iteration that ends the solve (the energies of Sec. 2.6 read it).
template <bool CACHE, bool FULL = false>
__device__ inline void scf_active_body(const ActiveArgs& a, unsigned lb, unsigned G, FdLds& fdl, double* sh,
                                       double* r, double* vls, double* xls) {
  ScfState* st = a.st;
  // the state as the launch found it, read before the first all-reduce: block 0
  // advances it after the last one, while other blocks may still be on their
  // way out of that all-reduce
  const int t = st->iter;
  // arrival counters: launches alternate between two banks; block 0 clears the
  // bank of the next launch (this launch does not touch it, the previous one
  // has ended)
  unsigned* bank = a.flags + ARRIVE_BANK * (unsigned)(t & 1);
  if (lb == 0 && threadIdx.x < ARRIVE_BANK)
    coherent_store_u32(a.flags + ARRIVE_BANK * (unsigned)((t + 1) & 1) + threadIdx.x, 0u);
  unsigned nred = 0;  // all-reduces of this launch so far
  // K and U_xc are formed with the active density only once More's weight is on;
  // in the iteration where it switches on they take a pass of their own
  const bool k_on = st->more_on != 0;
  const int more_on0 = st->more_on;
  const int64_t nchunk = a.nchunk;
  const double kT = a.kT;
  const double ikT = 1.0 / kT;
  const double mu_prev = st->mu;  // NaN on the first iteration
  const bool try_prev = mu_prev == mu_prev;
  const bool young = lb >= G / 2;  // the second half of the group (take_turn)
  // with CACHE each block owns at most one chunk (lb), otherwise chunks lb, lb+G, ...
#define FOR_CHUNKS(c)                                           \
  for (int64_t c = lb; c < nchunk; c += (CACHE ? nchunk : G))

  // 1. potential assembly (+ the Taylor sums of N at the previous mu).  Each
  // group's loads are issued a group ahead, so they are in flight while the
  // previous group is evaluated; the first group's overlap the load of the
  // I_{1/2} table into LDS.
  double pn[PG], pe[PG], ph[PG], pl[PG];
  auto fetch = [&](int64_t c, int q0) {
#pragma unroll
    for (int g = 0; g < PG; ++g) {
      const int64_t i = chunk_point(a, c, q0 + g);
      const int64_t ic = (FULL || i < a.ng) ? i : a.ng - 1;
      pn[g] = a.n_i[ic];
      pe[g] = a.Vie[ic];
      ph[g] = a.VH[ic];
      pl[g] = a.lap_i[ic];
    }
  };
  if ((int64_t)lb < nchunk) fetch(lb, 0);
  fd_lds_load(&fdl, a.fdt);
  __syncthreads();
  FOR_CHUNKS(c) {
    double acc[7] = {0.0, -INFINITY, -INFINITY, 0.0, 0.0, 0.0, 0.0};
    if (c != (int64_t)lb) fetch(c, 0);
#pragma unroll 1
  for (int q0 = 0; q0 < PPT; q0 += PG) {
      take_turn(q0 / PG, young);
      bool ok[PG];
      double n[PG], v[PG], lp[PG], vx[PG];
#pragma unroll
      for (int g = 0; g < PG; ++g) {
        ok[g] = FULL || chunk_point(a, c, q0 + g) < a.ng;
        n[g] = pn[g];
        v[g] = pe[g] + ph[g];
        lp[g] = pl[g];
      }
      if (q0 + PG < PPT) fetch(c, q0 + PG);
      if (a.xc) {
        vxc_group(n, vx);
      } else {
#pragma unroll
        for (int g = 0; g < PG; ++g) vx[g] = 0.0;
      }
#pragma unroll
      for (int g = 0; g < PG; ++g) {
        v[g] += vx[g];
        if (a.lam != 0.0) v[g] += -0.5 * a.lam * lp[g] * rsqrt_nr(n[g]);
        if (CACHE) {
          vls[(q0 + g) * SCF_THREADS + threadIdx.x] = v[g];
          xls[(q0 + g) * SCF_THREADS + threadIdx.x] = vx[g];
        } else if (ok[g]) {
          a.Vi[chunk_point(a, c, q0 + g)] = v[g];
        }
        acc[0] += ok[g] ? v[g] : 0.0;
        acc[1] = ok[g] ? fmax(acc[1], v[g]) : acc[1];
        acc[2] = ok[g] ? fmax(acc[2], -v[g]) : acc[2];
      }
      if (try_prev) {
        double x[PG], d[PG][4];
#pragma unroll
        for (int g = 0; g < PG; ++g) x[g] = (mu_prev - v[g]) * ikT;
        fd_group<3>(fdl, x, d);
#pragma unroll
        for (int g = 0; g < PG; ++g) {
          acc[3] += ok[g] ? d[g][0] : 0.0;
          acc[4] += ok[g] ? d[g][1] : 0.0;
          acc[5] += ok[g] ? d[g][2] : 0.0;
          acc[6] += ok[g] ? d[g][3] : 0.0;
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    block_reduce_n<7>(acc, 0x6u, sh);
    put_chunk_n<7>(acc, a.part, 0, nchunk, c);
  }
  grid_allreduce(a.part, nchunk, a.res, 0, try_prev ? 7 : 3, 0x6u, G, lb, bank, ++nred, a.err, r, sh);
  const double Vsum = r[0], Vmax = r[1], Vmin = -r[2];
  const double scale = a.dv * a.cn;  // N = scale * sum I_{1/2}
  double lo = Vmin + kT * a.eta0;
  double hi = Vmax + kT * a.eta0;
  double mu = mu_prev;
  const bool use_prev = try_prev && lo <= mu && mu <= hi;
  if (!use_prev) mu = Vsum / (double)a.ng + kT * a.eta0;

  // 2. the mu search; it counts the evaluations of N(mu)
  int it = 0;
  bool found = false, have_sums = false, spec = false;
  double N = 0.0, dN = 0.0;
  double D[6] = {0, 0, 0, 0, 0, 0};
  if (use_prev) {
    it = 1;
    N = scale * r[3];
    dN = scale * ikT * r[4];
    const double f = N - a.Ne;
    if (fabs(f) <= MU_TOL * a.Ne) {
      found = true;
    } else {
      if (f > 0.0)
        hi = mu;
      else
        lo = mu;
      // root z = (mu - mu_prev)/kT of g(z) = g0 + g1 z + g2 z^2 + g3 z^3, the
      // cubic Taylor model of ln N(mu) - ln N_e, by Newton from z = 0 (ln N is
      // nearly linear where N grows exponentially in mu, so the model holds
      // over shifts of several kT)
      const double u1 = r[4] / r[3], u2 = r[5] / r[3], u3 = r[6] / r[3];
      const double g0 = log(r[3]) - log(a.Ne / scale), g1 = u1, g2 = 0.5 * (u2 - u1 * u1),
                   g3 = (u3 - 3.0 * u1 * u2 + 2.0 * u1 * u1 * u1) / 6.0;
      double z = 0.0;
      for (int k = 0; k < 8; ++k) {
        const double gz = fma(z, fma(z, fma(z, g3, g2), g1), g0);
        const double gp = fma(z, fma(z, 3.0 * g3, 2.0 * g2), g1);
        const double s = gz / gp;
        z -= s;
        if (fabs(s) <= 1e-16 * (1.0 + fabs(z))) break;
      }
      double mn = mu + kT * z;
      // the model's error is of order z^4/24 (relative to N; bounded by the
      // model of N itself, whose derivatives in the non-degenerate limit all
      // equal N); when that is within MU_TOL the pass at the root forms the
      // active sums as well
      spec = z * z * z * z * (1.0 / 24.0) <= 0.5 * MU_TOL;
      if (!(lo < mn && mn < hi)) {
        mn = mu - (log(N) - log(a.Ne)) * N / dN;
        if (!(lo < mn && mn < hi)) mn = 0.5 * (lo + hi);
        spec = false;
      }
      mu = mn;
    }
  }
  while (!found && it < a.max_newton) {
    ++it;
    if (spec) {
      FOR_CHUNKS(c) chunk_sums<CACHE, true, FULL>(a, c, vls, xls, mu, ikT, fdl, sh, k_on, young);
      grid_allreduce(a.part, nchunk, a.res, 0, 8, 0x80u, G, lb, bank, ++nred, a.err, r, sh);
    } else {
      FOR_CHUNKS(c) chunk_sums<CACHE, false, FULL>(a, c, vls, xls, mu, ikT, fdl, sh, true, young);
      grid_allreduce(a.part, nchunk, a.res, 0, 2, 0u, G, lb, bank, ++nred, a.err, r, sh);
    }
    N = scale * r[0];
    dN = scale * ikT * r[1];
    const double f = N - a.Ne;
    if (fabs(f) <= MU_TOL * a.Ne) {
      found = true;
      if (spec) {
        have_sums = true;
        for (int k = 0; k < 6; ++k) D[k] = r[2 + k];
      }
      break;
    }
    if (f > 0.0)
      hi = mu;
    else
      lo = mu;
    // Newton on ln N(mu) = ln N_e (the step of Newton on N near the root)
    double mn = mu - (log(N) - log(a.Ne)) * N / dN;
    if (!(lo < mn && mn < hi)) mn = 0.5 * (lo + hi);
    if (fabs(mn - mu) <= 1e-15 * (fabs(mu) + kT)) {
      mu = mn;
      found = true;
      break;
    }
    spec = fabs(f) <= SPEC_NEWTON * a.Ne;
    mu = mn;
  }

  // 3. active density and the mixing reductions (unless the last pass formed them)
  if (!have_sums) {
    FOR_CHUNKS(c) chunk_sums<CACHE, true, FULL>(a, c, vls, xls, mu, ikT, fdl, sh, k_on, young);
    grid_allreduce(a.part, nchunk, a.res, 0, 8, 0x80u, G, lb, bank, ++nred, a.err, r, sh);
    for (int k = 0; k < 6; ++k) D[k] = r[2 + k];
  }
  const double DD = D[0], NN = D[1], NA = D[4], MX = D[5];
  double KK = D[2], UU = D[3];
  const double res = sqrt(DD / NN);
  // every block reaches the same verdict (the sums are identical in all of them)
  const bool last = res < a.tol || !(res == res) || !found || t + 1 >= a.max_iter;
  // More's weight switches on at the first iteration past the warm-up where
  // the active density is close (max |dn|/n_a within the trust bound) or mu
  // has settled (Sec. 2.5.2)
  int more = more_on0;
  if (a.mixing != ARCHE_MIX_FIXED && !more && t >= a.warmup &&
      (MX <= a.trust || fabs(mu - mu_prev) <= MU_SETTLED * kT))
    more = 1;
  if (more && !k_on && a.mixing == ARCHE_MIX_MORE && !last) {
    FOR_CHUNKS(c) chunk_sums<CACHE, true, FULL>(a, c, vls, xls, mu, ikT, fdl, sh, true, young);
    grid_allreduce(a.part, nchunk, a.res, 0, 8, 0x80u, G, lb, bank, ++nred, a.err, r, sh);
    KK = r[4];
    UU = r[5];
  }
  if (CACHE && last) {
    FOR_CHUNKS(c) {
      for (int q = 0; q < PPT; ++q) {
        const int64_t i = chunk_point(a, c, q);
        if (i < a.ng) a.Vi[i] = vls[q * SCF_THREADS + threadIdx.x];
      }
    }
  }
#undef FOR_CHUNKS

  if (lb == 0 && threadIdx.x == 0) {
    st->mu = mu;
    st->N = N;
    st->dN = dN;
    st->res = res;
    st->K = a.dv * KK;
    st->Uxc = a.dv * UU;
    st->Na = a.dv * NA;
    st->maxrel = MX;
    st->newton_last = it;
    st->newton_total += it;
    st->iter = t + 1;
    st->more_on = more;
    if (!found) st->mu_fail = 1;
    // raised by any block's bounded wait: read through the device-coherent path
    const bool bad = !(res == res) || !found || __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bad) st->err = 1;
    st->done = last || bad;
  }
}

// One system: the whole cooperative grid is the group.
template <bool CACHE, bool FULL>
__global__ void __launch_bounds__(SCF_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) k_scf_active(ActiveArgs a) {
  __shared__ double sh[RED_SH];
  __shared__ double r[8];
  __shared__ FdLds fdl;
  __shared__ double vls[CACHE ? PPT * SCF_THREADS : 1], xls[CACHE ? PPT * SCF_THREADS : 1];
  if (a.st->done) return;
  scf_active_body<CACHE, FULL>(a, blockIdx.x, gridDim.x, fdl, sh, r, vls, xls);
}

// Many systems in one cooperative launch: system s owns blocks
// [group_begin[s], group_begin[s+1]) (its group), converged systems drop out.
__global__ void __launch_bounds__(SCF_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_scf_active_batch(const ActiveArgs* __restrict__ args, const int* __restrict__ group_begin, int nsys) {
  __shared__ double sh[RED_SH];
  __shared__ double r[8];
  __shared__ FdLds fdl;
  __shared__ double vls[PPT * SCF_THREADS], xls[PPT * SCF_THREADS];
  int s = 0;
  while (s + 1 < nsys && group_begin[s + 1] <= (int)blockIdx.x) ++s;
  const ActiveArgs a = args[s];
  if (a.st->done) return;
  const unsigned lb = blockIdx.x - group_begin[s];
  const unsigned G = group_begin[s + 1] - group_begin[s];
  if ((int64_t)G >= a.nchunk)
    scf_active_body<true>(a, lb, G, fdl, sh, r, vls, xls);
  else
    scf_active_body<false>(a, lb, G, fdl, sh, r, vls, xls);
}

// U_vW = int (v_vW[n_i] - v_vW[n_a]) (n_i - n_a), v_vW[n] = -(lambda/2) lap(sqrt n)/sqrt n
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_uvw_partial(const ScfState* st, const double* n_i, const double* lap_i, const double* n_a,
              const double* lap_a, int64_t ng, double lam, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  if (st->done || !st->more_on) return;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) {
    const double ni = n_i[i], na = n_a[i];
    const double vi = -0.5 * lam * lap_i[i] / sqrt(ni);
    const double va = -0.5 * lam * lap_a[i] / sqrt(na);
    s += (vi - va) * (ni - na);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ inline void half_index(int64_t m, int Ny, int Nh, int& ix, int& iy, int& iz) {
  iz = (int)(m % Nh);
  int64_t r = m / Nh;
  iy = (int)(r % Ny);
  ix = (int)(r / Ny);
}

__device__ inline double box_k(int i, int N, double L) { return (double)(i <= N / 2 ? i : i - N) / L; }

// sum over the full box of |dn^|^2/(pi k^2) from the half spectrum (mirror terms doubled)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_uh_partial(const ScfState* st, const cplx* nhat_i, const cplx* nhat_a, GridInfo g, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  if (st->done) return;
  double s = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    const double kx = box_k(ix, g.N[0], g.L[0]), ky = box_k(iy, g.N[1], g.L[1]), kz = (double)iz / g.L[2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    if (k2 == 0.0) continue;
    const cplx d = csub(nhat_i[m], nhat_a[m]);
    const double wgt = (iz == 0 || 2 * iz == g.N[2]) ? 1.0 : 2.0;
    s += wgt * (d.x * d.x + d.y * d.y) / (PI * k2);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The state after this iteration into the host's pinned ring: 8-byte words with
// system-scope stores, so the host sees them once the iteration's event is done.
// The state after this iteration into the host's pinned ring, one 8-byte word
// per thread with system-scope stores (the host reads it once the iteration's
// event is done).  `copy` is the block's LDS copy of the state; every thread of
// the block calls this.
constexpr int STATE_WORDS = (int)(sizeof(ScfState) / 8);
static_assert(sizeof(ScfState) % 8 == 0 && STATE_WORDS <= ARCHE_BLOCK, "whole words, one per thread");
__device__ inline void state_to_ring(const MixWeightArgs& m, ScfState* copy) {
  if (threadIdx.x == 0) *copy = *m.st;
  __syncthreads();
  const int k = threadIdx.x;
  if (k < STATE_WORDS) {
    uint64_t* dst = (uint64_t*)(m.ring + (copy->iter - 1) % m.ring_n);
    __hip_atomic_store(dst + k, ((const uint64_t*)copy)[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Mixing weight (Sec. 2.5.2): w = U/(U+K) with U = U_H + U_xc + U_vW once the More
// weight is on, else w_fixed; clamped to [0, 0.995] and to at most W_MAX_DROP
// below the previous weight.  One block per system.  A converged (or failed)
// state skips the weight but still reaches the host's ring.
__device__ inline void mix_weight_body(const MixWeightArgs& m, double* sh, ScfState* copy) {
  ScfState* st = m.st;
  if (!st->done) {
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < m.nbh; t += blockDim.x) a += m.part_h[t];
    a = block_sum(a, sh);
    if (m.use_vw && st->more_on)
      for (int t = threadIdx.x; t < m.nbv; t += blockDim.x) b += m.part_v[t];
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
      st->UH = a / m.vol;
      st->Uvw = (m.use_vw && st->more_on) ? m.dv * b : 0.0;
      double w = m.w_fixed;
      if (st->more_on) {
        const double U = st->UH + st->Uxc + st->Uvw;
        w = U / (U + st->K);
        w = fmin(fmax(w, 0.0), 0.995);
        // at most W_MAX_DROP below the previous weight (st->w)
        if (m.bound_drop) w = fmax(w, st->w - W_MAX_DROP);
        if (!(w == w)) w = m.w_fixed;
      }
      st->w = w;
    }
  }
  if (m.ring) state_to_ring(m, copy);
}
__global__ void __launch_bounds__(ARCHE_BLOCK) k_mix_weight(MixWeightArgs m) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  __shared__ ScfState copy;
  mix_weight_body(m, sh, &copy);
}
__global__ void __launch_bounds__(ARCHE_BLOCK) k_mix_weight_batch(const MixWeightArgs* __restrict__ jobs) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  __shared__ ScfState copy;
  const MixWeightArgs m = jobs[blockIdx.x];
  mix_weight_body(m, sh, &copy);
}

// n^_o = n^_a + w (n^_i - n^_a) -> nhat_i;  tmp = n^_o / (pi k^2) (0 at k = 0).
// Once the solve is done n^_i stays and tmp = n^_i / (pi k^2), so that the
// C2R that follows reproduces V_H[n_i] instead of overwriting it.
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_spec_mix(const ScfState* st, cplx* nhat_i, const cplx* nhat_a, cplx* tmp, GridInfo g) {
  const bool done = st->done;
  const double w = st->w;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    const double kx = box_k(ix, g.N[0], g.L[0]), ky = box_k(iy, g.N[1], g.L[1]), kz = (double)iz / g.L[2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    const cplx a = nhat_a[m];
    const cplx o = done ? nhat_i[m] : cadd(a, cscale(csub(nhat_i[m], a), w));
    if (!done) nhat_i[m] = o;
    tmp[m] = k2 > 0.0 ? cscale(o, 1.0 / (PI * k2)) : cplx{0.0, 0.0};
  }
}

// n_o = n_a + w (n_i - n_a) -> n_i;  sq = sqrt(n_o)   (block bid of nb)
__device__ inline void real_mix_body(const RealMixArgs& r, unsigned bid, unsigned nb) {
  if (r.st->done) {
    // the unfused iteration's later transforms run anyway: sq = sqrt(n_i) keeps
    // lap sqrt(n_i) as it is (the fused passes stop by themselves instead)
    if (r.sqrt_when_done)
      for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < r.ng; i += (int64_t)nb * blockDim.x)
        r.sq[i] = sqrt(r.n_i[i]);
    return;
  }
  const double w = r.st->w;
  for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < r.ng; i += (int64_t)nb * blockDim.x) {
    const double na = r.n_a[i];
    const double no = na + w * (r.n_i[i] - na);
    r.n_i[i] = no;
    r.sq[i] = sqrt(no);
  }
}
__global__ void __launch_bounds__(ARCHE_BLOCK) k_real_mix(RealMixArgs r) { real_mix_body(r, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_real_mix_batch(const RealMixArgs* __restrict__ jobs, const int* __restrict__ bbeg, int njobs) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bbeg[mid] <= (int)blockIdx.x)
      lo = mid;
    else
      hi = mid - 1;
  }
  const RealMixArgs r = jobs[lo];
  real_mix_body(r, blockIdx.x - (unsigned)bbeg[lo], (unsigned)(bbeg[lo + 1] - bbeg[lo]));
}

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_sqrt(const ScfState* st, int need_more, const double* in, double* out, int64_t ng) {
  if (st && (st->done || (need_more && !st->more_on))) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = sqrt(in[i]);
}

// s^ -> -(2 pi |k|)^2 s^
__global__ void __launch_bounds__(ARCHE_BLOCK) k_spec_lap(cplx* s, GridInfo g) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    const double kx = box_k(ix, g.N[0], g.L[0]), ky = box_k(iy, g.N[1], g.L[1]), kz = (double)iz / g.L[2];
    const double q2 = 4.0 * PI * PI * (kx * kx + ky * ky + kz * kz);
    s[m] = cscale(s[m], -q2);
  }
}

// n^ -> n^/(pi k^2), 0 at k = 0 (Hartree, Sec. 2.3)
__global__ void __launch_bounds__(ARCHE_BLOCK) k_spec_hartree(const cplx* nhat, cplx* out, GridInfo g) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    const double kx = box_k(ix, g.N[0], g.L[0]), ky = box_k(iy, g.N[1], g.L[1]), kz = (double)iz / g.L[2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    out[m] = k2 > 0.0 ? cscale(nhat[m], 1.0 / (PI * k2)) : cplx{0.0, 0.0};
  }
}

// Energy sums at the converged (eta = (mu - V_i)/kT, n_a) of Sec. 2.6:
// 0 sum f0, 1 sum p0, 2 sum n eps_xc, 3 sum n (v_xc - eps_xc), 4 sum n V^ie, 5 sum n
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_energy_real(const ScfState* st, const double* Vi, const double* Vie, const FdTables* fdt, int64_t ng,
              double kT, double cn, double pc, int xc, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  const double mu = st->mu;
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) {
    const double eta = (mu - Vi[i]) / kT;
    const double ip = fd_eval_order(fdt, 1, eta);
    const double i32 = fd_eval_order(fdt, 2, eta);
    const double n = cn * ip;
    const double p0 = pc * i32;
    s[0] += n * kT * eta - p0;
    s[1] += p0;
    if (xc) {
      double v;
      const double e = lda_xc(n, v);
      s[2] += n * e;
      s[3] += n * (v - e);
    }
    s[4] += n * Vie[i];
    s[5] += n;
  }
  for (int q = 0; q < 6; ++q) {
    double v = block_sum(s[q], sh);
    if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = v;
  }
}

// sum over the full box of w(k) |f^(k)|^2 with w = 1/(pi k^2) (kind 0) or (2 pi k)^2 (kind 1)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_spec_norm(const cplx* f, GridInfo g, int kind, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  double s = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    const double kx = box_k(ix, g.N[0], g.L[0]), ky = box_k(iy, g.N[1], g.L[1]), kz = (double)iz / g.L[2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    if (k2 == 0.0) continue;
    const double wgt = (iz == 0 || 2 * iz == g.N[2]) ? 1.0 : 2.0;
    const double a2 = f[m].x * f[m].x + f[m].y * f[m].y;
    s += wgt * a2 * (kind == 0 ? 1.0 / (PI * k2) : 4.0 * PI * PI * k2);
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(ARCHE_BLOCK) k_finish_sums(const double* part, int nblk, int nsum, double* out) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  for (int q = 0; q < nsum; ++q) {
    double v = 0.0;
    for (int t = threadIdx.x; t < nblk; t += blockDim.x) v += part[(size_t)q * nblk + t];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[q] = v;
  }
}

__global__ void __launch_bounds__(ARCHE_BLOCK) k_fill(double* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

__global__ void k_state_init(ScfState* st, unsigned* flags, int nflags, int* err, double mu0) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ScfState z{};
    z.mu = mu0;
    *st = z;
    *err = 0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nflags; i += gridDim.x * blockDim.x) flags[i] = 0u;
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + ARCHE_BLOCK - 1) / ARCHE_BLOCK;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (unsigned)b;
}

#define HIP_TRY(x)                         \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return e_;       \
  } while (0)

}  // namespace

size_t scf_part_offset(const arche_ctx* c) {
  const int64_t nchunk = (c->g.ng + SCF_CHUNK - 1) / SCF_CHUNK;
  return 16 * (size_t)std::max<int64_t>(nchunk, c->coop_blocks);
}

int red_blocks(int64_t n) {
  int64_t b = (n + 4 * ARCHE_BLOCK - 1) / (4 * ARCHE_BLOCK);
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t finish_sums(const double* partials, int nblk, int nsum, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(ARCHE_BLOCK), 0, s, partials, nblk, nsum, out);
  return hipGetLastError();
}

// Fermi-Dirac tables: one upload per device, kept for the life of the process.
const FdTables* fd_tables_device(int device) {
  static std::mutex mtx;
  static FdTables* per_dev[64] = {nullptr};
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mtx);
  if (!per_dev[device]) {
    FdTables h;
    for (int j = 0; j < 3; ++j) {
      for (int k = 0; k < FD_KSER; ++k) h.ser[j][k] = FD_SER[j][k];
      for (int k = 0; k < FD_KASY; ++k) h.asy[j][k] = FD_ASY[j][k];
      for (int i = 0; i < FD_NINT; ++i)
        for (int k = 0; k < FD_NCOEF; ++k) h.poly[j][i][k] = FD_POLY[j][i][k];
    }
    FdTables* d = nullptr;
    if (hipMalloc(&d, sizeof(FdTables)) != hipSuccess) return nullptr;
    if (hipMemcpy(d, &h, sizeof(FdTables), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    per_dev[device] = d;
  }
  return per_dev[device];
}

hipError_t scf_reset_state(arche_ctx* c, double mu0) {
  hipLaunchKernelGGL(k_state_init, dim3(4), dim3(ARCHE_BLOCK), 0, c->stream, c->state, c->bar, SCF_BAR_WORDS,
                     c->err_d, mu0);
  return hipGetLastError();
}

// lap = del^2 sqrt(n) through the spectral Laplacian: inverse(-(2 pi k)^2 forward(sqrt n))
hipError_t scf_vw_laplacian(arche_ctx* c, const double* n, double* lap) {
  const GridInfo& g = c->g;
  hipLaunchKernelGGL(k_sqrt, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)nullptr, 0, n,
                     c->rtmp, g.ng);
  HIP_TRY(hipGetLastError());
  HIP_TRY(fft_r2c(&c->plan, c->rtmp, c->ctmp, 1.0, g.dv, c->stream));
  hipLaunchKernelGGL(k_spec_lap, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->ctmp, g);
  HIP_TRY(hipGetLastError());
  return fft_c2r(&c->plan, c->ctmp, lap, 1.0 / g.vol, c->stream);
}

hipError_t scf_sqrt_spectrum(arche_ctx* c, const double* n, cplx* out) {
  const GridInfo& g = c->g;
  hipLaunchKernelGGL(k_sqrt, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)nullptr, 0, n,
                     c->rtmp, g.ng);
  HIP_TRY(hipGetLastError());
  return fft_r2c(&c->plan, c->rtmp, out, 1.0, g.dv, c->stream);
}

// From the input density n_i: n^_i, V_H[n_i], lap(sqrt n_i).
static hipError_t prepare_input(arche_ctx* c) {
  const GridInfo& g = c->g;
  HIP_TRY(fft_r2c(&c->plan, c->n_i, c->nhat_i, 1.0, g.dv, c->stream));
  hipLaunchKernelGGL(k_spec_hartree, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->nhat_i, c->ctmp, g);
  HIP_TRY(hipGetLastError());
  HIP_TRY(fft_c2r(&c->plan, c->ctmp, c->VH, 1.0 / g.vol, c->stream));
  if (c->p.lambda_vw != 0.0) return scf_vw_laplacian(c, c->n_i, c->lap_i);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, c->lap_i, g.ng, 0.0);
  return hipGetLastError();
}

hipError_t scf_initial_uniform(arche_ctx* c) {
  const GridInfo& g = c->g;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, c->n_i, g.ng, c->Ne / g.vol);
  HIP_TRY(hipGetLastError());
  return prepare_input(c);
}

hipError_t scf_prepare_input(arche_ctx* c) { return prepare_input(c); }

// Blocks of the cooperative SCF launch: all co-resident, at most two per CU, and
// no more than the grid needs.  Fixed for a given device and grid, so the
// reduction order (and the result) is reproducible.
int scf_coop_blocks(int64_t ng) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int per_cu = 1 << 20;
  for (const void* k : {(const void*)k_scf_active<true, false>, (const void*)k_scf_active<false, false>,
                        (const void*)k_scf_active<true, true>, (const void*)k_scf_active<false, true>}) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, SCF_THREADS, 0) != hipSuccess) return 0;
    per_cu = std::min(per_cu, n);
  }
  int64_t b = std::min<int64_t>((int64_t)per_cu * cus, 2 * (int64_t)cus);
  b = std::min<int64_t>(b, (ng + 4 * ARCHE_BLOCK - 1) / (4 * ARCHE_BLOCK));
  return (int)std::max<int64_t>(b, 1);
}

static ActiveArgs active_args(const arche_ctx* c) {
  const GridInfo& g = c->g;
  const arche_params& p = c->p;
  ActiveArgs a{};
  a.Vie = c->Vie;
  a.VH = c->VH;
  a.lap_i = c->lap_i;
  a.n_i = c->n_i;
  a.Vi = c->Vi;
  a.n_a = c->n_a;
  a.st = c->state;
  a.part = c->partials;
  a.res = c->sums + 32;
  a.flags = c->bar;
  a.err = c->err_d;
  a.fdt = c->fdt;
  a.ng = g.ng;
  a.nchunk = (g.ng + SCF_CHUNK - 1) / SCF_CHUNK;
  a.dv = g.dv;
  a.kT = p.kT;
  a.cn = std::pow(2.0 * p.kT, 1.5) / (2.0 * PI * PI);
  a.Ne = c->Ne;
  a.lam = p.lambda_vw;
  a.xc = p.xc;
  a.eta0 = c->eta0;
  a.tol = p.scf_tol;
  a.mixing = p.mixing;
  a.warmup = p.more_warmup;
  a.trust = p.more_trust;
  a.max_newton = 200;
  a.max_iter = p.scf_max_iter;
  return a;
}

static void push_pass(std::vector<IterStep>& v, int slot, const FftPass& a) {
  IterStep st{};
  st.slot = slot;
  st.kind = STEP_FFT;
  st.fft = a;
  st.nblocks = a.nblocks;
  v.push_back(st);
}
static void push_dual(std::vector<IterStep>& v, int slot, const FftPass& a, const FftPass& b) {
  IterStep st{};
  st.slot = slot;
  st.kind = STEP_FFT;
  st.fft = a;
  st.fft2 = b;
  st.dual = 1;
  st.nblocks = a.nblocks + b.nblocks;
  v.push_back(st);
}

static void push_fft(std::vector<IterStep>& v, int slot, const FftPass* ps) {
  for (int i = 0; i < 3; ++i) {
    IterStep st{};
    st.slot = slot + i;
    st.kind = STEP_FFT;
    st.fft = ps[i];
    st.nblocks = ps[i].nblocks;
    v.push_back(st);
  }
}

// The rest of an SCF iteration with the spectral and pointwise steps fused into
// the FFT passes (fft.h): R2C(n_a) also sums U_H; [More + vW: R2C(sqrt n_a) with
// the Laplacian on store, C2R that sums U_vW instead of storing]; the weight;
// C2R of n_o^/(pi k^2) that forms n_o^ from n^_a and n^_i on load; R2C of
// sqrt(n_o) that forms n_o on load, Laplacian on store, C2R -> lap sqrt(n_o).
// Every pass stops once the state's done flag is raised.
void scf_build_iteration(arche_ctx* c) {
  if (c->iter_built) return;
  c->active = active_args(c);
  c->steps.clear();
  c->fused = fft_fusable(&c->plan);
  c->iter_built = true;
  if (!c->fused) return;
  const GridInfo& g = c->g;
  const arche_params& p = c->p;
  const bool vw = p.lambda_vw != 0.0;
  const bool more = p.mixing == ARCHE_MIX_MORE;
  // With plane passes (N_y = N_z) independent transforms share launches (below).
  const bool pair = fft_plane_fusable(&c->plan);
  // Where the x length has it (rt), the Laplacian of sqrt n goes forward along
  // x, is multiplied, and comes back along x at once (x pass MODE 4), so the C2R
  // that follows starts at its plane pass.
  const bool rt = pair && fft_x_roundtrip(g.N[0]);
  // with More + vW on such grids the U_H x pass runs re-tiled beside the U_vW
  // plane pass, in fewer blocks (fewer U_H partials)
  const bool uh_wide = rt && more && vw;
  const int nbh = uh_wide ? fft_x_blocks_wide(&c->plan) : fft_x_blocks(&c->plan);
  const int nbv = fft_z_blocks(&c->plan);
  double* part_h = c->partials + scf_part_offset(c);
  double* part_v = part_h + nbh;
  // With More and vW the SCF kernel sums U_vW's v_vW[n_i] part and leaves
  // (n_i - n_a)/sqrt(n_a) in lap_a (free during the solve) for the C2R pass
  // that sums the v_vW[n_a] part.
  if (more && vw) c->active.uvw_w = c->lap_a;
  FftFuse f{};
  f.w = &c->state->w;
  f.n_i = c->n_i;
  f.n_a = c->n_a;
  f.lap_i = c->lap_i;
  f.nhat_i = c->nhat_i;
  f.lam = p.lambda_vw;
  f.L[0] = g.L[0];
  f.L[1] = g.L[1];
  f.L[2] = g.L[2];
  f.partials = part_h;
  f.stop = &c->state->done;
  // Paired launches: the plane passes of R2C(n_a) and R2C(sqrt n_a); with the
  // round trip, the U_H x pass with the U_vW plane pass (the round trip alone
  // before them; without it the x passes run one after the other); the Hartree
  // C2R's plane pass with that of R2C(sqrt n_o), which then works in ctmp2.
  FftPass ps[3];
  fft_r2c_passes(&c->plan, c->n_a, c->nhat_a, 1.0, g.dv, FUSE_NONE, R2C_OUT_UH, f, ps);
  if (pair && more && vw) {
    FftPass pb[3], pu[3];
    fft_r2c_passes(&c->plan, c->n_a, c->ctmp, 1.0, g.dv, R2C_IN_SQRT, R2C_OUT_LAP, f, pb);
    if (rt) pb[2].mode = 4;
    push_dual(c->steps, SLOT_NHAT_A, ps[0], pb[0]);
    FftFuse fv = f;
    fv.partials = part_v;
    fv.uvw_w = c->lap_a;
    fft_c2r_passes(&c->plan, c->ctmp, c->ctmp, nullptr, 1.0 / g.vol, FUSE_NONE, C2R_OUT_UVW, fv, pu);
    if (rt) {
      push_pass(c->steps, SLOT_LAP_A + 2, pb[2]);
      push_dual(c->steps, SLOT_UVW + 2, ps[2], pu[2]);
    } else {
      push_dual(c->steps, SLOT_NHAT_A + 2, ps[2], pb[2]);
      push_pass(c->steps, SLOT_UVW, pu[0]);
      push_pass(c->steps, SLOT_UVW + 2, pu[2]);
    }
  } else {
    push_fft(c->steps, SLOT_NHAT_A, ps);
  }
  if (more && vw && !pair) {
    fft_r2c_passes(&c->plan, c->n_a, c->ctmp, 1.0, g.dv, R2C_IN_SQRT, R2C_OUT_LAP, f, ps);
    push_fft(c->steps, SLOT_LAP_A, ps);
    FftFuse fv = f;
    fv.partials = part_v;
    fv.uvw_w = c->lap_a;
    fft_c2r_passes(&c->plan, c->ctmp, c->ctmp, nullptr, 1.0 / g.vol, FUSE_NONE, C2R_OUT_UVW, fv, ps);
    push_fft(c->steps, SLOT_UVW, ps);
  }
  IterStep w{};
  w.slot = SLOT_WEIGHT;
  w.kind = STEP_WEIGHT;
  w.nblocks = 1;
  w.mw = MixWeightArgs{c->state, part_h, nbh, part_v, nbv, (int)(more && vw), g.vol, g.dv, p.w_fixed, (int)more,
                       c->state_host, ARCHE_RING};
  c->steps.push_back(w);
  if (pair && vw) {
    FftPass pe[3], pf[3];
    fft_c2r_passes(&c->plan, c->nhat_a, c->ctmp, c->VH, 1.0 / g.vol, C2R_IN_MIX, FUSE_NONE, f, pe);
    fft_r2c_passes(&c->plan, c->n_a, c->ctmp2, 1.0, g.dv, R2C_IN_MIX_SQRT, R2C_OUT_LAP, f, pf);
    fft_c2r_passes(&c->plan, c->ctmp2, c->ctmp2, c->lap_i, 1.0 / g.vol, FUSE_NONE, FUSE_NONE, f, ps);
    if (rt) {
      // the Hartree x pass beside R2C(sqrt n_o)'s plane pass; the Laplacian's
      // round trip; the two C2R plane passes (-> V_H, -> lap sqrt(n_o)) together
      pf[2].mode = 4;
      push_dual(c->steps, SLOT_HARTREE, pe[0], pf[0]);
      push_pass(c->steps, SLOT_SQRT_O + 2, pf[2]);
      push_dual(c->steps, SLOT_HARTREE + 2, pe[2], ps[2]);
      return;
    }
    push_pass(c->steps, SLOT_HARTREE, pe[0]);
    push_dual(c->steps, SLOT_HARTREE + 2, pe[2], pf[0]);
    push_pass(c->steps, SLOT_SQRT_O + 2, pf[2]);
    push_pass(c->steps, SLOT_LAP_O, ps[0]);
    push_pass(c->steps, SLOT_LAP_O + 2, ps[2]);
    return;
  }
  fft_c2r_passes(&c->plan, c->nhat_a, c->ctmp, c->VH, 1.0 / g.vol, C2R_IN_MIX, FUSE_NONE, f, ps);
  push_fft(c->steps, SLOT_HARTREE, ps);
  if (vw) {
    fft_r2c_passes(&c->plan, c->n_a, c->ctmp, 1.0, g.dv, R2C_IN_MIX_SQRT, R2C_OUT_LAP, f, ps);
    push_fft(c->steps, SLOT_SQRT_O, ps);
    fft_c2r_passes(&c->plan, c->ctmp, c->ctmp, c->lap_i, 1.0 / g.vol, FUSE_NONE, FUSE_NONE, f, ps);
    push_fft(c->steps, SLOT_LAP_O, ps);
  } else {
    IterStep r{};
    r.slot = SLOT_REAL_MIX;
    r.kind = STEP_REAL_MIX;
    r.nblocks = scf_real_mix_blocks(g.ng);
    r.rm = RealMixArgs{c->state, c->n_i, c->n_a, c->rtmp, g.ng, 0};
    c->steps.push_back(r);
  }
}

unsigned scf_real_mix_blocks(int64_t ng) { return grid_for(ng); }

hipError_t scf_step_launch(const IterStep& st, hipStream_t s) {
  if (st.kind == STEP_FFT) return st.dual ? fft_dual_launch(st.fft, st.fft2, s) : fft_pass_launch(st.fft, s);
  if (st.kind == STEP_WEIGHT)
    hipLaunchKernelGGL(k_mix_weight, dim3(1), dim3(ARCHE_BLOCK), 0, s, st.mw);
  else
    hipLaunchKernelGGL(k_real_mix, dim3(st.nblocks), dim3(ARCHE_BLOCK), 0, s, st.rm);
  return hipGetLastError();
}

// the unfused sequence, for grids without compile-time FFT plans
static hipError_t scf_iteration_rest_plain(arche_ctx* c) {
  const GridInfo& g = c->g;
  const arche_params& p = c->p;
  const bool vw = p.lambda_vw != 0.0;
  const bool more = p.mixing == ARCHE_MIX_MORE;
  // n^_a
  HIP_TRY(fft_r2c(&c->plan, c->n_a, c->nhat_a, 1.0, g.dv, c->stream));
  const int nbr = red_blocks(g.ng);
  const int nbh = red_blocks(g.nh);
  double* part_h = c->partials + scf_part_offset(c);
  double* part_v = part_h + nbh;
  if (more && vw) {
    // lap(sqrt n_a) for the von Weizsaecker part of U
    hipLaunchKernelGGL(k_sqrt, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)c->state, 1,
                       c->n_a, c->rtmp, g.ng);
    HIP_TRY(hipGetLastError());
    HIP_TRY(fft_r2c(&c->plan, c->rtmp, c->ctmp, 1.0, g.dv, c->stream));
    hipLaunchKernelGGL(k_spec_lap, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->ctmp, g);
    HIP_TRY(hipGetLastError());
    HIP_TRY(fft_c2r(&c->plan, c->ctmp, c->lap_a, 1.0 / g.vol, c->stream));
    hipLaunchKernelGGL(k_uvw_partial, dim3(nbr), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)c->state, c->n_i,
                       c->lap_i, c->n_a, c->lap_a, g.ng, p.lambda_vw, part_v);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_uh_partial, dim3(nbh), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)c->state, c->nhat_i,
                     c->nhat_a, g, part_h);
  HIP_TRY(hipGetLastError());
  const MixWeightArgs mw{c->state, part_h, nbh, part_v, nbr, (int)(more && vw), g.vol, g.dv, p.w_fixed, (int)more,
                         c->state_host, ARCHE_RING};
  hipLaunchKernelGGL(k_mix_weight, dim3(1), dim3(ARCHE_BLOCK), 0, c->stream, mw);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_spec_mix, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)c->state,
                     c->nhat_i, c->nhat_a, c->ctmp, g);
  HIP_TRY(hipGetLastError());
  HIP_TRY(fft_c2r(&c->plan, c->ctmp, c->VH, 1.0 / g.vol, c->stream));
  const RealMixArgs rm{c->state, c->n_i, c->n_a, c->rtmp, g.ng, 1};
  hipLaunchKernelGGL(k_real_mix, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, rm);
  HIP_TRY(hipGetLastError());
  if (vw) {
    HIP_TRY(fft_r2c(&c->plan, c->rtmp, c->ctmp, 1.0, g.dv, c->stream));
    hipLaunchKernelGGL(k_spec_lap, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->ctmp, g);
    HIP_TRY(hipGetLastError());
    HIP_TRY(fft_c2r(&c->plan, c->ctmp, c->lap_i, 1.0 / g.vol, c->stream));
  }
  return hipSuccess;
}

bool scf_plain_launch(const arche_ctx* c) { return c->p.exclusive_device && g_live_contexts.load() == 1; }

hipError_t scf_iteration(arche_ctx* c) {
  scf_build_iteration(c);
  void* args[] = {&c->active};
  const bool cache = c->active.nchunk <= c->coop_blocks;
  {
    ProfScope prof(PROF_SCF_ACTIVE, c->stream);
    // The kernel's all-reduces need every block resident at once.  The grid is
    // the occupancy-sized count of one kernel alone on the device.  A
    // cooperative launch guarantees residency.  When the caller has declared
    // the device its own (exclusive_device) and this context is the only one
    // in the process, nothing else can hold CUs while waiting on the kernel
    // (other kernels finish by themselves, then the rest of the grid is
    // dispatched), and a plain launch saves the ~20 us a cooperative launch
    // spends around the kernel.  Waits are bounded in any case (a time-out
    // raises the error flag instead of hanging).
    const bool full = c->active.ng % SCF_CHUNK == 0;
    const void* kern = cache ? (full ? (const void*)k_scf_active<true, true> : (const void*)k_scf_active<true, false>)
                             : (full ? (const void*)k_scf_active<false, true> : (const void*)k_scf_active<false, false>);
    if (scf_plain_launch(c)) {
      HIP_TRY(hipLaunchKernel(kern, dim3(c->coop_blocks), dim3(SCF_THREADS), args, 0, c->stream));
    } else {
      HIP_TRY(hipLaunchCooperativeKernel(kern, dim3(c->coop_blocks), dim3(SCF_THREADS), args, 0, c->stream));
    }
  }
  if (!c->fused) return scf_iteration_rest_plain(c);
  for (const IterStep& st : c->steps) HIP_TRY(scf_step_launch(st, c->stream));
  return hipSuccess;
}

int scf_batch_capacity() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_scf_active_batch, SCF_THREADS, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

hipError_t scf_active_batch_launch(const ActiveArgs* args, const int* group_begin, int nsys, int nblocks,
                                   hipStream_t s) {
  void* kargs[] = {&args, &group_begin, &nsys};
  ProfScope prof(PROF_SCF_ACTIVE, s);
  return hipLaunchCooperativeKernel((const void*)k_scf_active_batch, dim3(nblocks), dim3(SCF_THREADS), kargs, 0, s);
}

hipError_t scf_weight_batch_launch(const MixWeightArgs* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mix_weight_batch, dim3(njobs), dim3(ARCHE_BLOCK), 0, s, jobs);
  return hipGetLastError();
}

hipError_t scf_real_mix_batch_launch(const RealMixArgs* jobs, const int* bbeg, int njobs, unsigned nblocks,
                                     hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_real_mix_batch, dim3(nblocks), dim3(ARCHE_BLOCK), 0, s, jobs, bbeg, njobs);
  return hipGetLastError();
}

// out: 0 F_TF, 1 K_e, 2 F_xc, 3 P_xc, 4 int n V^ie, 5 int n, 6 E_H, 7 F_vW, 8 P_TF
hipError_t scf_energies(arche_ctx* c, double* out) {
  const GridInfo& g = c->g;
  const arche_params& p = c->p;
  const double cn = std::pow(2.0 * p.kT, 1.5) / (2.0 * PI * PI);
  const double pc = (2.0 * std::sqrt(2.0) / (3.0 * PI * PI)) * std::pow(p.kT, 2.5);
  const int nbr = red_blocks(g.ng);
  hipLaunchKernelGGL(k_energy_real, dim3(nbr), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)c->state, c->Vi,
                     c->Vie, c->fdt, g.ng, p.kT, cn, pc, p.xc, c->partials);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(c->partials, nbr, 6, c->sums, c->stream));
  HIP_TRY(fft_r2c(&c->plan, c->n_a, c->nhat_a, 1.0, g.dv, c->stream));
  const int nbh = red_blocks(g.nh);
  double* part2 = c->partials + 6 * (size_t)nbr;
  hipLaunchKernelGGL(k_spec_norm, dim3(nbh), dim3(ARCHE_BLOCK), 0, c->stream, (const cplx*)c->nhat_a, g, 0, part2);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(part2, nbh, 1, c->sums + 6, c->stream));
  if (p.lambda_vw != 0.0) {
    hipLaunchKernelGGL(k_sqrt, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, (const ScfState*)nullptr, 0,
                       c->n_a, c->rtmp, g.ng);
    HIP_TRY(hipGetLastError());
    HIP_TRY(fft_r2c(&c->plan, c->rtmp, c->ctmp, 1.0, g.dv, c->stream));
    double* part3 = part2 + nbh;
    hipLaunchKernelGGL(k_spec_norm, dim3(nbh), dim3(ARCHE_BLOCK), 0, c->stream, (const cplx*)c->ctmp, g, 1, part3);
    HIP_TRY(hipGetLastError());
    HIP_TRY(finish_sums(part3, nbh, 1, c->sums + 7, c->stream));
  }
  double h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(h, c->sums, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  out[0] = g.dv * h[0];
  out[1] = 1.5 * g.dv * h[1];
  out[2] = g.dv * h[2];
  out[3] = h[3] / (double)g.ng;
  out[4] = g.dv * h[4];
  out[5] = g.dv * h[5];
  out[6] = 0.5 * h[6] / g.vol;
  out[7] = p.lambda_vw != 0.0 ? 0.5 * p.lambda_vw * h[7] / g.vol : 0.0;
  out[8] = h[1] / (double)g.ng;
  return hipSuccess;
}
