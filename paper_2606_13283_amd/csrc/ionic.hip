// Position-dependent kernels: structure factor and ionic field (Sec. 2.4), Ewald
// ion-ion energy and forces (Sec. 2.6.3), electron-ion forces and pressure term
// (Sec. 2.6.5), and the one-center shell profile (Sec. 2.5.1).
//
// Spectra live on the half box m_z in [0, N_z/2].  A full-box sum is the sum over
// the stored points plus, for 0 < m_z < N_z/2, the mirror point -m.  The mirror of
// a point whose x or y index is the Nyquist index N/2 is not -k: the box keeps
// only +N/2.  Writing k~ for k with its Nyquist components negated, the mirror
// contributes the conjugate of the term at k~.  So every kernel here carries
// S+(m) = S(k_m) and S-(m) = S(k~_m) (equal unless m has a Nyquist component),
// and the Hermitian part of S that a real field sees is (S+ + S-)/2.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "arche_internal.h"

namespace {

constexpr double PI = 3.14159265358979323846;

__device__ inline void half_index(int64_t m, int Ny, int Nh, int& ix, int& iy, int& iz) {
  iz = (int)(m % Nh);
  int64_t r = m / Nh;
  iy = (int)(r % Ny);
  ix = (int)(r / Ny);
}

__device__ inline int box_m(int i, int N) { return i <= N / 2 ? i : i - N; }

// phase tables exp(-2 pi i k_m x / L) for box index m (axis a), z only m <= Nz/2,
// one row per atom in species order: row q holds atom order[q]
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_phases(const double* pos, const int* __restrict__ order, int n_atoms, GridInfo g, cplx* phx, cplx* phy, cplx* phz) {
  const int64_t total = (int64_t)n_atoms * (g.N[0] + g.N[1] + g.Nh);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e / (g.N[0] + g.N[1] + g.Nh);
    int r = (int)(e - q * (g.N[0] + g.N[1] + g.Nh));
    int axis, i;
    if (r < g.N[0]) {
      axis = 0;
      i = r;
    } else if (r < g.N[0] + g.N[1]) {
      axis = 1;
      i = r - g.N[0];
    } else {
      axis = 2;
      i = r - g.N[0] - g.N[1];
    }
    const int64_t j = order[q];
    const int m = axis == 2 ? i : box_m(i, g.N[axis]);
    double f = pos[j * 3 + axis] / g.L[axis];
    f -= floor(f);
    double th = (double)m * f;
    th -= rint(th);  // exp(-2 pi i th) is 1-periodic in th
    double s, c;
    sincospi(2.0 * th, &s, &c);
    cplx v{c, -s};
    if (axis == 0)
      phx[q * g.N[0] + i] = v;
    else if (axis == 1)
      phy[q * g.N[1] + i] = v;
    else
      phz[q * g.Nh + i] = v;
  }
}

// S+_s(m) = sum_{j in s} P_j(k_m), S-_s(m) = sum_{j in s} P_j(k~_m), atoms
// sorted by species.  P_j = px py pz splits into the factors without a Nyquist
// index (a) and those with one (b); S+ sums a b = P, S- sums a conj(b).  The
// half box is walked as rows (ix, iy) by z indices: each lane takes one row and
// SZ_CZ consecutive z indices from iz0 = SZ_CZ blockIdx.y.  Atoms go in
// batches of SZ_AB: the batch's z phases are staged in LDS (read by the whole
// wave at one address), its row phases per lane in registers, and the next
// batch's loads are in flight while one is summed.
//   MIRROR = false: every row; S+ everywhere, and S- where it differs from S+
//     only by the z Nyquist index (iz = N_z/2: S- sums px py conj(pz)) on rows
//     without a Nyquist x or y index, S- = S+ elsewhere on those rows.
//   MIRROR = true: the rows with a Nyquist x or y index (ix = N_x/2 for even
//     N_x: rows 0..N_y-1 of this launch; iy = N_y/2 for even N_y: the others,
//     each row once); S- with those row factors conjugated.
constexpr int SZ_CZ = 8;
constexpr int SZ_AB = 8;
__device__ inline void nyq_row_of(int r, const GridInfo& g, int& ix, int& iy) {
  const int nrx = (g.N[0] % 2 == 0) ? g.N[1] : 0;
  if (r < nrx) {
    ix = g.N[0] / 2;
    iy = r;
  } else {
    const int r2 = r - nrx;
    iy = g.N[1] / 2;
    ix = (g.N[0] % 2 == 0 && r2 >= g.N[0] / 2) ? r2 + 1 : r2;
  }
}
template <bool MIRROR>
__device__ inline void structure_rows_body(const cplx* __restrict__ phx, const cplx* __restrict__ phy,
                                           const cplx* __restrict__ phz, const int* __restrict__ sp_begin, int ns,
                                           const GridInfo& g, int rows, unsigned bx, cplx* __restrict__ Sp,
                                           cplx* __restrict__ Sm, cplx (*zl)[SZ_AB * SZ_CZ]) {
  const int lane = threadIdx.x;
  const int row = (int)bx * 64 + lane;
  const int iz0 = (int)blockIdx.y * SZ_CZ;
  const bool live = row < rows;
  const int rr = live ? row : rows - 1;
  int ix, iy;
  if (MIRROR) {
    nyq_row_of(rr, g, ix, iy);
  } else {
    ix = rr / g.N[1];
    iy = rr - ix * g.N[1];
  }
  const bool nx = 2 * ix == g.N[0], ny = 2 * iy == g.N[1];
  const bool nyq_row = nx || ny;
  // the z Nyquist index inside this chunk (uniform), else -1
  const int tN = (g.N[2] % 2 == 0 && g.N[2] / 2 >= iz0 && g.N[2] / 2 < iz0 + SZ_CZ) ? g.N[2] / 2 - iz0 : -1;
  for (int s = 0; s < ns; ++s) {
    cplx acc[SZ_CZ], accN{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < SZ_CZ; ++t) acc[t] = cplx{0.0, 0.0};
    const int qb = sp_begin[s], qe = sp_begin[s + 1];
    // loads of the batch at q0 (atoms past qe clamp to qe - 1; their terms are skipped)
    cplx xn[SZ_AB], yn[SZ_AB], zn;
    auto fetch = [&](int q0) {
#pragma unroll
      for (int u = 0; u < SZ_AB; ++u) {
        const int64_t q = min(q0 + u, qe - 1);
        xn[u] = phx[q * g.N[0] + ix];
        yn[u] = phy[q * g.N[1] + iy];
      }
      const int64_t q = min(q0 + lane / SZ_CZ, qe - 1);
      zn = phz[q * g.Nh + min(iz0 + lane % SZ_CZ, g.Nh - 1)];
    };
    static_assert(SZ_AB * SZ_CZ == 64, "one z phase per lane");
    if (qb < qe) fetch(qb);
    int buf = 0;
    for (int q0 = qb; q0 < qe; q0 += SZ_AB, buf ^= 1) {
      zl[buf][lane] = zn;
      cplx xc[SZ_AB], yc[SZ_AB];
#pragma unroll
      for (int u = 0; u < SZ_AB; ++u) {
        xc[u] = MIRROR && nx ? cconj(xn[u]) : xn[u];
        yc[u] = MIRROR && ny ? cconj(yn[u]) : yn[u];
      }
      __syncthreads();
      if (q0 + SZ_AB < qe) fetch(q0 + SZ_AB);
      const int nu = min(SZ_AB, qe - q0);
#pragma unroll
      for (int u = 0; u < SZ_AB; ++u) {
        if (u < nu) {
          const cplx pxy = cmul(xc[u], yc[u]);
          const cplx* z = zl[buf] + u * SZ_CZ;
#pragma unroll
          for (int t = 0; t < SZ_CZ; ++t) {
            const cplx zt = z[t];
            acc[t].x = fma(pxy.x, zt.x, fma(-pxy.y, zt.y, acc[t].x));
            acc[t].y = fma(pxy.x, zt.y, fma(pxy.y, zt.x, acc[t].y));
          }
          if (tN >= 0) {  // pxy conj(pz) at the z Nyquist index
            const cplx zt = z[tN];
            accN.x = fma(pxy.x, zt.x, fma(pxy.y, zt.y, accN.x));
            accN.y = fma(-pxy.x, zt.y, fma(pxy.y, zt.x, accN.y));
          }
        }
        // keeps the compiler from hoisting the next atoms' LDS reads (registers)
        asm volatile("" ::: "memory");
      }
    }
    __syncthreads();  // the next species reuses the buffers
    if (live) {
      const int64_t m0 = ((int64_t)ix * g.N[1] + iy) * g.Nh;
      cplx* sp = Sp + (int64_t)s * g.nh + m0;
      cplx* sm = Sm + (int64_t)s * g.nh + m0;
#pragma unroll
      for (int t = 0; t < SZ_CZ; ++t) {
        const int iz = iz0 + t;
        if (iz < g.Nh) {
          if (!MIRROR) sp[iz] = acc[t];
          if (MIRROR == nyq_row && t != tN) sm[iz] = acc[t];
        }
      }
      if (MIRROR == nyq_row && tN >= 0) sm[iz0 + tN] = accN;
    }
  }
}

// One launch: blocks [0, main_blocks) walk every row (MIRROR = false), the
// others the rows with a Nyquist x or y index (MIRROR = true), concurrently.
__global__ void __launch_bounds__(64)
k_structure_rows(const cplx* __restrict__ phx, const cplx* __restrict__ phy, const cplx* __restrict__ phz,
                 const int* __restrict__ sp_begin, int ns, GridInfo g, unsigned main_blocks, int nyq_rows,
                 cplx* __restrict__ Sp, cplx* __restrict__ Sm) {
  __shared__ cplx zl[2][SZ_AB * SZ_CZ];
  if (blockIdx.x < main_blocks)
    structure_rows_body<false>(phx, phy, phz, sp_begin, ns, g, g.N[0] * g.N[1], blockIdx.x, Sp, Sm, zl);
  else
    structure_rows_body<true>(phx, phy, phz, sp_begin, ns, g, nyq_rows, blockIdx.x - main_blocks, Sp, Sm, zl);
}

__device__ inline void kvec(int ix, int iy, int iz, const GridInfo& g, double k[3]) {
  k[0] = (double)box_m(ix, g.N[0]) / g.L[0];
  k[1] = (double)box_m(iy, g.N[1]) / g.L[1];
  k[2] = (double)iz / g.L[2];
}

__device__ inline double form_factor(double q, double Z, double rc) {
  return -Z * cos(2.0 * PI * q * rc) / (PI * q * q);
}

// Tabulated non-Coulomb part D_s at q > 0: the cubic through the nodes i-1..i+2
// around x = q/dq (local cubic Lagrange; node -1 mirrors node 1, D_s being even
// in q).  Returns D_s(q) and, in *dd, its derivative in q.
__device__ inline double ff_table_eval(const double* f, double dq, double q, double* dd) {
  const double x = q / dq;
  const int i = (int)floor(x);
  const double t = x - (double)i;
  const double fm = f[i == 0 ? 1 : i - 1], f0 = f[i], f1 = f[i + 1], f2 = f[i + 2];
  const double tp = t + 1.0, tm = t - 1.0, tmm = t - 2.0;
  const double lm = -t * tm * tmm / 6.0, l0 = tp * tm * tmm / 2.0, l1 = -tp * t * tmm / 2.0, l2 = tp * t * tm / 6.0;
  // derivatives of the four basis cubics in t
  const double dm = -(3.0 * t * t - 6.0 * t + 2.0) / 6.0;
  const double d0 = (3.0 * t * t - 4.0 * t - 1.0) / 2.0;
  const double d1 = -(3.0 * t * t - 2.0 * t - 2.0) / 2.0;
  const double d2 = (3.0 * t * t - 1.0) / 6.0;
  *dd = (fm * dm + f0 * d0 + f1 * d1 + f2 * d2) / dq;
  return fm * lm + f0 * l0 + f1 * l1 + f2 * l2;
}

// V_s(q) for q > 0 (Sec. 2.4, eq. iepseudo)
__device__ inline double species_ff(const SpeciesInfo& sp, int s, double q) {
  if (!sp.ff) return form_factor(q, sp.Z[s], sp.rc[s]);
  double dd;
  return ff_table_eval(sp.ff + (int64_t)s * sp.ff_len, sp.ff_dq, q, &dd) - sp.Z[s] / (PI * q * q);
}

// dV_s/dq for q > 0 (k2 = q^2)
__device__ inline double species_ff_dq(const SpeciesInfo& sp, int s, double q, double k2) {
  if (!sp.ff) {
    const double a = 2.0 * PI * q * sp.rc[s];
    return sp.Z[s] * (2.0 * PI * sp.rc[s] * sin(a) / k2 + 2.0 * cos(a) / (k2 * q)) / PI;
  }
  double dd;
  (void)ff_table_eval(sp.ff + (int64_t)s * sp.ff_len, sp.ff_dq, q, &dd);
  return dd + 2.0 * sp.Z[s] / (PI * k2 * q);
}

// SZ+- = sum_s Z_s S+-_s ; V^ie^(m) = sum_s V_s(|k|) (S+_s + S-_s)/2 (Hermitian part)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_vie_hat(const cplx* Sp, const cplx* Sm, SpeciesInfo sp, GridInfo g, cplx* SZp, cplx* SZm, cplx* vhat) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    double k[3];
    kvec(ix, iy, iz, g, k);
    const double q = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    cplx zp{0, 0}, zm{0, 0}, v{0, 0};
    for (int s = 0; s < sp.ns; ++s) {
      const cplx a = Sp[(int64_t)s * g.nh + m], b = Sm[(int64_t)s * g.nh + m];
      zp = cadd(zp, cscale(a, sp.Z[s]));
      zm = cadd(zm, cscale(b, sp.Z[s]));
      if (q > 0.0) v = cadd(v, cscale(cadd(a, b), 0.5 * species_ff(sp, s, q)));
    }
    SZp[m] = zp;
    SZm[m] = zm;
    vhat[m] = v;
  }
}

// Ewald real-space pairs (minimum image): per-atom forces and half the pair
// energy.  One block per atom j; its threads take the partners l in a fixed
// stride and the block sums them in a fixed order.
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_ewald_pairs(const double* pos, const double* Zat, int n, GridInfo g, double alpha, double* F, double* Uj) {
  __shared__ double sh[(ARCHE_BLOCK / 64) * 4];
  const int j = blockIdx.x;
  const double xj = pos[3 * j], yj = pos[3 * j + 1], zj = pos[3 * j + 2];
  double acc[4] = {0, 0, 0, 0};  // fx, fy, fz, u
  const double c2 = 2.0 * alpha / sqrt(PI);
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    if (l == j) continue;
    double d[3] = {xj - pos[3 * l], yj - pos[3 * l + 1], zj - pos[3 * l + 2]};
    for (int a = 0; a < 3; ++a) d[a] -= g.L[a] * rint(d[a] / g.L[a]);
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = sqrt(r2);
    const double zz = Zat[j] * Zat[l];
    const double e = erfc(alpha * r) / r;
    acc[3] += 0.5 * zz * e;
    const double coef = zz * (e + c2 * exp(-alpha * alpha * r2)) / r2;
    acc[0] += coef * d[0];
    acc[1] += coef * d[1];
    acc[2] += coef * d[2];
  }
  block_reduce_n<4>(acc, 0u, sh);
  if (threadIdx.x == 0) {
    F[3 * j] = acc[0];
    F[3 * j + 1] = acc[1];
    F[3 * j + 2] = acc[2];
    Uj[j] = acc[3];
  }
}

// full-box sum of V_alpha |S_Z|^2 (k != 0)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_ewald_recip(const cplx* SZp, const cplx* SZm, GridInfo g, double alpha, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  double s = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    double k[3];
    kvec(ix, iy, iz, g, k);
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 == 0.0) continue;
    const double va = exp(-PI * PI * k2 / (alpha * alpha)) / (PI * k2);
    const cplx a = SZp[m];
    double t = a.x * a.x + a.y * a.y;
    if (iz != 0 && 2 * iz != g.N[2]) {
      const cplx b = SZm[m];
      t += b.x * b.x + b.y * b.y;
    }
    s += va * t;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Force weights per species: W+-_s(m) = V_s(|k|) conj(n^(m)) + Z_s V_alpha(|k|) conj(SZ+-(m))
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_force_weights(const cplx* nhat, const cplx* SZp, const cplx* SZm, SpeciesInfo sp, GridInfo g, double alpha,
                cplx* Wp, cplx* Wm) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    double k[3];
    kvec(ix, iy, iz, g, k);
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const cplx n = cconj(nhat[m]);
    const cplx zp = cconj(SZp[m]), zm = cconj(SZm[m]);
    for (int s = 0; s < sp.ns; ++s) {
      cplx wp{0, 0}, wm{0, 0};
      if (k2 > 0.0) {
        const double q = sqrt(k2);
        const double vs = species_ff(sp, s, q);
        const double va = sp.Z[s] * exp(-PI * PI * k2 / (alpha * alpha)) / (PI * k2);
        wp = cadd(cscale(n, vs), cscale(zp, va));
        wm = cadd(cscale(n, vs), cscale(zm, va));
      }
      Wp[(int64_t)s * g.nh + m] = wp;
      Wm[(int64_t)s * g.nh + m] = wm;
    }
  }
}

// Phase tables transposed for the force kernel: phT = [x: N_x][y: N_y][z: N_h]
// rows of n_atoms values in species order (the order of the phase tables), so
// that lanes taking consecutive atoms read consecutive values.
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_phases_T(const cplx* __restrict__ phx, const cplx* __restrict__ phy, const cplx* __restrict__ phz, int n, GridInfo g,
           cplx* __restrict__ phT) {
  const int64_t total = (int64_t)n * (g.N[0] + g.N[1] + g.Nh);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n;
    const int64_t q = e - i * n;
    cplx v;
    if (i < g.N[0])
      v = phx[q * g.N[0] + i];
    else if (i < g.N[0] + g.N[1])
      v = phy[q * g.N[1] + (i - g.N[0])];
    else
      v = phz[q * g.Nh + (i - g.N[0] - g.N[1])];
    phT[e] = v;
  }
}

// F_j = -(2 pi/|Omega|) sum over the full box of Im(W(k) exp(-2 pi i k.r_j)) k.
// The half box is walked as rows (ix, iy) by z indices.  A block is one wave:
// its lanes take 64 atoms (species order), it walks the rows of one row block
// and, CZ z indices at a time, all of N_h.  Rows go in batches of FRB: the
// batch's W_s (the same for the whole wave) is staged in LDS, the row phases px,
// py per lane in registers, and the next batch's loads are in flight while one
// is summed; the CZ z phases of the lane's atom stay in registers.  Full-box
// weighting: 2 for 0 < iz < N_z/2 (the mirror -k), 1 at iz = 0 and the z
// Nyquist index; on a row with a Nyquist x or y index the mirror is k~ instead,
// with its own weight W-(m) and the Nyquist phase factors conjugated.
constexpr int FRB = 8;
constexpr int FORCE_CZ = 16;
template <int CZ>
__device__ inline void force_rows_chunk(const cplx* __restrict__ W, const cplx* __restrict__ WM,
                                        const cplx* __restrict__ xT, const cplx* __restrict__ yT,
                                        const cplx* __restrict__ zT, int n, int qc, const GridInfo& g, int r0,
                                        int r1, int iz0, double* f, cplx (*wl)[FRB * FORCE_CZ]) {
  constexpr int PER = (FRB * CZ + 63) / 64;
  const int lane = threadIdx.x;
  cplx pz[CZ];
#pragma unroll
  for (int t = 0; t < CZ; ++t) pz[t] = zT[(int64_t)(iz0 + t) * n + qc];
  // loads of the batch of rows at rb (rows past r1 clamp to r1 - 1; skipped)
  cplx wn[PER], xn[FRB], yn[FRB];
  auto fetch = [&](int rb) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = lane + 64 * p;
      if (e < FRB * CZ) {
        const int r = min(rb + e / CZ, r1 - 1);
        wn[p] = W[(int64_t)r * g.Nh + iz0 + e % CZ];
      }
    }
    int ix = rb / g.N[1], iy = rb - ix * g.N[1];
#pragma unroll
    for (int u = 0; u < FRB; ++u) {
      xn[u] = xT[(int64_t)ix * n + qc];
      yn[u] = yT[(int64_t)iy * n + qc];
      // the next row, unless this was the block's last
      if (rb + u + 1 < r1 && ++iy == g.N[1]) {
        iy = 0;
        ++ix;
      }
    }
  };
  fetch(r0);
  int buf = 0;
  for (int rb = r0; rb < r1; rb += FRB, buf ^= 1) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int e = lane + 64 * p;
      if (e < FRB * CZ) wl[buf][e] = wn[p];
    }
    cplx xc[FRB], yc[FRB];
#pragma unroll
    for (int u = 0; u < FRB; ++u) {
      xc[u] = xn[u];
      yc[u] = yn[u];
    }
    __syncthreads();
    if (rb + FRB < r1) fetch(rb + FRB);
    int ix = rb / g.N[1], iy = rb - ix * g.N[1];
#pragma unroll
    for (int u = 0; u < FRB; ++u) {
      const int r = rb + u;
      if (r < r1) {
        const cplx pxy = cmul(xc[u], yc[u]);
        const bool nx = 2 * ix == g.N[0], ny = 2 * iy == g.N[1];
        const double kx = (double)box_m(ix, g.N[0]) / g.L[0], ky = (double)box_m(iy, g.N[1]) / g.L[1];
        const cplx* w = wl[buf] + u * CZ;
        if (!(nx || ny)) {
          double sr = 0.0, sz = 0.0;
#pragma unroll
          for (int t = 0; t < CZ; ++t) {
            const int iz = iz0 + t;
            const cplx wv = w[t];
            const double Px = pxy.x * pz[t].x - pxy.y * pz[t].y;
            const double Py = pxy.x * pz[t].y + pxy.y * pz[t].x;
            const double im = (iz != 0 && 2 * iz != g.N[2] ? 2.0 : 1.0) * (wv.x * Py + wv.y * Px);
            sr += im;
            sz += im * (double)iz;
          }
          f[0] += sr * kx;
          f[1] += sr * ky;
          f[2] += sz / g.L[2];
        } else {
          const cplx pxym = cmul(nx ? cconj(xc[u]) : xc[u], ny ? cconj(yc[u]) : yc[u]);
          const cplx* wm = WM + (int64_t)r * g.Nh + iz0;
          double sp = 0.0, szp = 0.0, sm = 0.0, szm = 0.0;
#pragma unroll
          for (int t = 0; t < CZ; ++t) {
            const int iz = iz0 + t;
            const cplx wv = w[t];
            const double Px = pxy.x * pz[t].x - pxy.y * pz[t].y;
            const double Py = pxy.x * pz[t].y + pxy.y * pz[t].x;
            const double im = wv.x * Py + wv.y * Px;
            sp += im;
            szp += im * (double)iz;
            if (iz != 0 && 2 * iz != g.N[2]) {
              const cplx wmv = wm[t];
              const double Qx = pxym.x * pz[t].x - pxym.y * pz[t].y;
              const double Qy = pxym.x * pz[t].y + pxym.y * pz[t].x;
              const double im2 = wmv.x * Qy + wmv.y * Qx;
              sm += im2;
              szm += im2 * (double)iz;
            }
          }
          f[0] += sp * kx + sm * (nx ? -kx : kx);
          f[1] += sp * ky + sm * (ny ? -ky : ky);
          f[2] += (szp + szm) / g.L[2];
        }
      }
      if (++iy == g.N[1]) {
        iy = 0;
        ++ix;
      }
      // keeps the compiler from hoisting the next rows' LDS reads (registers)
      asm volatile("" ::: "memory");
    }
  }
  __syncthreads();  // the next chunk reuses the buffers
}

__global__ void __launch_bounds__(64)
k_force_rows(const cplx* __restrict__ Wp, const cplx* __restrict__ Wm, const cplx* __restrict__ phT,
             const int* __restrict__ order, const int* __restrict__ spec, int n, GridInfo g, int rows_per_block,
             double* __restrict__ part /*[row blocks][n][3]*/) {
  __shared__ cplx wl[2][FRB * FORCE_CZ];
  const int q = (int)blockIdx.x * 64 + (int)threadIdx.x;
  const bool live = q < n;
  const int qc = live ? q : n - 1;
  const int j = order[qc];
  const int sj = spec[j];
  const int s_lo = spec[order[blockIdx.x * 64]];
  const int s_hi = spec[order[min((int)blockIdx.x * 64 + 63, n - 1)]];
  const int rows = g.N[0] * g.N[1];
  const int r0 = (int)blockIdx.y * rows_per_block;
  const int r1 = min(r0 + rows_per_block, rows);
  const cplx* xT = phT;
  const cplx* yT = phT + (int64_t)g.N[0] * n;
  const cplx* zT = yT + (int64_t)g.N[1] * n;
  double f[3] = {0.0, 0.0, 0.0};
  double fs[3];
  for (int s = s_lo; s <= s_hi; ++s) {
    // every lane runs every species of its group (the LDS batches are shared);
    // a lane keeps the sums of its own species
    const cplx* W = Wp + (int64_t)s * g.nh;
    const cplx* WM = Wm + (int64_t)s * g.nh;
    fs[0] = fs[1] = fs[2] = 0.0;
    int iz0 = 0;
    for (; iz0 + FORCE_CZ <= g.Nh; iz0 += FORCE_CZ)
      force_rows_chunk<FORCE_CZ>(W, WM, xT, yT, zT, n, qc, g, r0, r1, iz0, fs, wl);
    for (; iz0 + 4 <= g.Nh; iz0 += 4) force_rows_chunk<4>(W, WM, xT, yT, zT, n, qc, g, r0, r1, iz0, fs, wl);
    for (; iz0 < g.Nh; ++iz0) force_rows_chunk<1>(W, WM, xT, yT, zT, n, qc, g, r0, r1, iz0, fs, wl);
    if (sj == s) {
      f[0] = fs[0];
      f[1] = fs[1];
      f[2] = fs[2];
    }
  }
  if (live) {
#pragma unroll
    for (int a = 0; a < 3; ++a) part[((int64_t)blockIdx.y * n + j) * 3 + a] = f[a];
  }
}

// F_j = -(2 pi/|Omega|) sum_chunks part + F^pp_j, in fixed chunk order: one
// wave per component, its lanes taking the chunks in a fixed stride
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_force_finish(const double* part, int nchunk, int n_atoms, double vol, const double* Fpp, double* F) {
  const int q = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= n_atoms * 3) return;  // whole waves leave together
  double s = 0.0;
  for (int c = lane; c < nchunk; c += 64) s += part[(int64_t)c * n_atoms * 3 + q];
  s = wave_sum(s);
  if (lane == 0) F[q] = -2.0 * PI / vol * s + Fpp[q];
}

// P_ie spectral part: full-box sum of Re(conj(n^) |k| V_s'(|k|) S_s)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_pressure_ie(const cplx* nhat, const cplx* Sp, const cplx* Sm, SpeciesInfo sp, GridInfo g, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  double acc = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    double k[3];
    kvec(ix, iy, iz, g, k);
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 == 0.0) continue;
    const double q = sqrt(k2);
    const bool interior = iz != 0 && 2 * iz != g.N[2];
    const cplx n = nhat[m];
    for (int s = 0; s < sp.ns; ++s) {
      const double dv = species_ff_dq(sp, s, q, k2);
      const cplx b = Sp[(int64_t)s * g.nh + m];
      double t = n.x * b.x + n.y * b.y;  // Re(conj(n) S+)
      if (interior) {
        const cplx c = Sm[(int64_t)s * g.nh + m];
        t += n.x * c.x + n.y * c.y;
      }
      acc += q * dv * t;
    }
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Shells whose sum |S_Z|^2 is below SHELL_CUT x (shell size) x sum_j Z_j^2 get no
// one-center profile (the fit there is ill-conditioned).
constexpr double SHELL_CUT = 1e-12;

// one-center profile per shell: g = sum Re(n^ conj SZ) / sum |SZ|^2 over the
// full box.  One wave per shell: its lanes take the shell's points in a fixed
// stride and the wave sums them in a fixed order.
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_shell_profile(const cplx* nhat, const cplx* SZp, const cplx* SZm, const int* perm, const int* off, int nshell,
                GridInfo g, double sumZ2, double* gsh) {
  const int s = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= nshell) return;  // whole waves leave together
  double num = 0.0, den = 0.0, cnt = 0.0;
  for (int q = off[s] + lane; q < off[s + 1]; q += 64) {
    const int64_t m = perm[q];
    const int iz = (int)(m % g.Nh);
    const cplx n = nhat[m];
    const cplx a = SZp[m];
    num += n.x * a.x + n.y * a.y;
    den += a.x * a.x + a.y * a.y;
    cnt += 1.0;
    if (iz != 0 && 2 * iz != g.N[2]) {
      const cplx b = SZm[m];
      num += n.x * b.x + n.y * b.y;
      den += b.x * b.x + b.y * b.y;
      cnt += 1.0;
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  cnt = wave_sum(cnt);
  if (lane == 0) gsh[s] = den > SHELL_CUT * cnt * sumZ2 ? num / den : 0.0;
}

// n^_i(m) = g(shell(m)) (SZ+(m) + SZ-(m))/2
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_one_center_hat(const double* gsh, const int* shell_of, const cplx* SZp, const cplx* SZm, GridInfo g, cplx* out) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    const double v = 0.5 * gsh[shell_of[m]];
    out[m] = cscale(cadd(SZp[m], SZm[m]), v);
  }
}

// floor at f0 and the two integrals (raw, floored)
__global__ void __launch_bounds__(ARCHE_BLOCK) k_floor(double* n, int64_t ng, double f0, double* part) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  double raw = 0.0, fl = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) {
    double v = n[i];
    raw += v;
    v = fmax(v, f0);
    n[i] = v;
    fl += v;
  }
  raw = block_sum(raw, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = raw;
  fl = block_sum(fl, sh);
  if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = fl;
}

// b <- a - b on a half spectrum
__global__ void __launch_bounds__(ARCHE_BLOCK) k_spec_sub(const cplx* a, cplx* b, int64_t nh) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = csub(a[i], b[i]);
}

__global__ void __launch_bounds__(ARCHE_BLOCK) k_fill_ni(double* n, int64_t ng, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) n[i] = v;
}

__global__ void __launch_bounds__(ARCHE_BLOCK) k_scale(double* n, int64_t ng, double s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) n[i] *= s;
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + ARCHE_BLOCK - 1) / ARCHE_BLOCK;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (unsigned)b;
}

#define HIP_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)


// Stress tensor sums over the full box (Sec. 2.6), six components each in the
// order xx, yy, zz, yz, xz, xy, from the half box: a stored point m stands for
// k and, off the k_z = 0 and Nyquist planes, for the mirror -k~ (k~ = k with its
// Nyquist x / y components negated), whose k_mu k_nu is that of k~.
//   ee: |n^|^2/(pi k^2) k_mu k_nu / k^2           (k != 0)
//   vw: |s^|^2 k_mu k_nu
//   ie: sum_s Re(conj(n^) S_s) V_s'(|k|) k_mu k_nu / |k|   (k != 0)
//   pm: V_alpha |S_Z|^2 (pi^2/alpha^2 + 1/k^2) k_mu k_nu   (k != 0)
// Block partials: part[(term * 6 + c) * nblk + block].
__device__ inline void kk6(const double* k, double w, double* o) {
  o[0] += w * k[0] * k[0];
  o[1] += w * k[1] * k[1];
  o[2] += w * k[2] * k[2];
  o[3] += w * k[1] * k[2];
  o[4] += w * k[0] * k[2];
  o[5] += w * k[0] * k[1];
}

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_stress_recip(const cplx* nhat, const cplx* shat, const cplx* Sp, const cplx* Sm, const cplx* SZp, const cplx* SZm,
               SpeciesInfo sp, GridInfo g, double alpha, double* part) {
  __shared__ double sh[(ARCHE_BLOCK / 64) * 8];
  double acc[24];
#pragma unroll
  for (int q = 0; q < 24; ++q) acc[q] = 0.0;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    double k[3];
    kvec(ix, iy, iz, g, k);
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const bool interior = iz != 0 && 2 * iz != g.N[2];
    const double kt[3] = {2 * ix == g.N[0] ? -k[0] : k[0], 2 * iy == g.N[1] ? -k[1] : k[1], k[2]};
    if (shat) {
      const cplx sv = shat[m];
      const double w = sv.x * sv.x + sv.y * sv.y;
      kk6(k, w, acc + 6);
      if (interior) kk6(kt, w, acc + 6);
    }
    if (k2 == 0.0) continue;
    const double q = sqrt(k2);
    const cplx n = nhat[m];
    const double wee = (n.x * n.x + n.y * n.y) / (PI * k2 * k2);
    kk6(k, wee, acc);
    if (interior) kk6(kt, wee, acc);
    double wp = 0.0, wm = 0.0;
    for (int s = 0; s < sp.ns; ++s) {
      const double dv = species_ff_dq(sp, s, q, k2) / q;
      const cplx b = Sp[(int64_t)s * g.nh + m];
      wp += dv * (n.x * b.x + n.y * b.y);  // Re(conj(n) S+)
      if (interior) {
        const cplx c = Sm[(int64_t)s * g.nh + m];
        wm += dv * (n.x * c.x + n.y * c.y);
      }
    }
    kk6(k, wp, acc + 12);
    if (interior) kk6(kt, wm, acc + 12);
    const double va = exp(-PI * PI * k2 / (alpha * alpha)) / (PI * k2) * (PI * PI / (alpha * alpha) + 1.0 / k2);
    const cplx zp = SZp[m];
    kk6(k, va * (zp.x * zp.x + zp.y * zp.y), acc + 18);
    if (interior) {
      const cplx zm = SZm[m];
      kk6(kt, va * (zm.x * zm.x + zm.y * zm.y), acc + 18);
    }
  }
  for (int b = 0; b < 3; ++b) {
    block_reduce_n<8>(acc + 8 * b, 0u, sh);
    if (threadIdx.x == 0)
      for (int q = 0; q < 8; ++q) part[(size_t)(8 * b + q) * gridDim.x + blockIdx.x] = acc[8 * b + q];
    __syncthreads();
  }
}

// Ewald real-space pair tensor, per atom j: (1/2) sum_{l != j} Z_j Z_l
// [erfc(alpha d)/d + 2 alpha/sqrt(pi) exp(-alpha^2 d^2)] d_mu d_nu / d^2 (minimum image),
// six components per atom [j][6]; one block per atom, as k_ewald_pairs
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_ewald_pair_stress(const double* pos, const double* Zat, int n, GridInfo g, double alpha, double* out) {
  __shared__ double sh[(ARCHE_BLOCK / 64) * 6];
  const int j = blockIdx.x;
  const double xj = pos[3 * j], yj = pos[3 * j + 1], zj = pos[3 * j + 2];
  const double c2 = 2.0 * alpha / sqrt(PI);
  double o[6] = {0, 0, 0, 0, 0, 0};
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    if (l == j) continue;
    double d[3] = {xj - pos[3 * l], yj - pos[3 * l + 1], zj - pos[3 * l + 2]};
    for (int a = 0; a < 3; ++a) d[a] -= g.L[a] * rint(d[a] / g.L[a]);
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = sqrt(r2);
    const double coef = 0.5 * Zat[j] * Zat[l] * (erfc(alpha * r) / r + c2 * exp(-alpha * alpha * r2)) / r2;
    kk6(d, coef, o);
  }
  block_reduce_n<6>(o, 0u, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) out[(size_t)q * n + j] = o[q];
}

}  // namespace

double ewald_alpha(const arche_ctx* c) {
  if (c->p.ewald_alpha > 0.0) return c->p.ewald_alpha;
  double kc = 1e300, rc = 1e300;
  for (int a = 0; a < 3; ++a) {
    kc = std::min(kc, c->g.N[a] / (2.0 * c->g.L[a]));
    rc = std::min(rc, c->g.L[a] / 2.0);
  }
  return std::sqrt(PI * kc / rc);
}

hipError_t ionic_structure(arche_ctx* c) {
  const GridInfo& g = c->g;
  hipLaunchKernelGGL(k_phases, dim3(grid_for((int64_t)c->n_atoms * (g.N[0] + g.N[1] + g.Nh))), dim3(ARCHE_BLOCK), 0,
                     c->stream, c->pos, c->sp_order, c->n_atoms, g, c->phx, c->phy, c->phz);
  HIP_TRY(hipGetLastError());
  const int rows = g.N[0] * g.N[1];
  const unsigned nzc = (unsigned)((g.Nh + SZ_CZ - 1) / SZ_CZ);
  const int nrx = (g.N[0] % 2 == 0) ? g.N[1] : 0;
  const int nry = (g.N[1] % 2 == 0) ? g.N[0] - (g.N[0] % 2 == 0 ? 1 : 0) : 0;
  const unsigned mb = (unsigned)((rows + 63) / 64), nb = (unsigned)((nrx + nry + 63) / 64);
  hipLaunchKernelGGL(k_structure_rows, dim3(mb + nb, nzc), dim3(64), 0, c->stream, c->phx, c->phy, c->phz,
                     c->sp_begin, c->n_species, g, mb, nrx + nry, c->Sp, c->Sm);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_vie_hat, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->Sp, c->Sm, c->sp, g, c->SZp,
                     c->SZm, c->ctmp);
  HIP_TRY(hipGetLastError());
  return fft_c2r(&c->plan, c->ctmp, c->Vie, 1.0 / g.vol, c->stream);
}

// U3 = {U_pp, U_pm, U_je}; also leaves F^pp in c->fpp (device)
hipError_t ionic_ewald(arche_ctx* c, double* U3, double alpha) {
  const GridInfo& g = c->g;
  const int n = c->n_atoms;
  double* Uj = c->partials;
  hipLaunchKernelGGL(k_ewald_pairs, dim3(n), dim3(ARCHE_BLOCK), 0, c->stream, c->pos,
                     c->Zatom, n, g, alpha, c->fpp, Uj);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(Uj, n, 1, c->sums, c->stream));
  const int nbh = red_blocks(g.nh);
  double* part = c->partials + n;
  hipLaunchKernelGGL(k_ewald_recip, dim3(nbh), dim3(ARCHE_BLOCK), 0, c->stream, c->SZp, c->SZm, g, alpha, part);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(part, nbh, 1, c->sums + 1, c->stream));
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, c->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  U3[0] = h[0];
  U3[1] = 0.5 / g.vol * h[1] - alpha / std::sqrt(PI) * c->sumZ2;
  U3[2] = -PI * c->Q * c->Q / (2.0 * alpha * alpha * g.vol);
  return hipSuccess;
}

// Row blocks of the force kernel: about 4096 waves in all (atom groups of 64 x
// row blocks), *rows_per_block rows each.
static int force_row_blocks(const arche_ctx* c, int* rows_per_block) {
  const int64_t rows = (int64_t)c->g.N[0] * c->g.N[1];
  const int64_t groups = (c->n_atoms + 63) / 64;
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(rows, 4096 / groups));
  const int64_t rpb = (rows + want - 1) / want;
  *rows_per_block = (int)rpb;
  return (int)((rows + rpb - 1) / rpb);
}

// forces (device [n][3]) from the converged spectrum nhat; needs ionic_ewald first (F^pp)
hipError_t ionic_forces(arche_ctx* c, const cplx* nhat, double* forces_dev) {
  const GridInfo& g = c->g;
  const double alpha = ewald_alpha(c);
  hipLaunchKernelGGL(k_force_weights, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, nhat, c->SZp, c->SZm,
                     c->sp, g, alpha, c->Wp, c->Wm);
  HIP_TRY(hipGetLastError());
  const int n = c->n_atoms;
  hipLaunchKernelGGL(k_phases_T, dim3(grid_for((int64_t)n * (g.N[0] + g.N[1] + g.Nh))), dim3(ARCHE_BLOCK), 0, c->stream,
                     c->phx, c->phy, c->phz, n, g, c->phT);
  HIP_TRY(hipGetLastError());
  int rpb = 0;
  const int nrb = force_row_blocks(c, &rpb);
  hipLaunchKernelGGL(k_force_rows, dim3((unsigned)((n + 63) / 64), (unsigned)nrb), dim3(64), 0, c->stream, c->Wp, c->Wm,
                     c->phT, c->sp_order, c->spec_d, n, g, rpb, c->fpart);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_force_finish, dim3((3 * n + ARCHE_BLOCK / 64 - 1) / (ARCHE_BLOCK / 64)), dim3(ARCHE_BLOCK), 0,
                     c->stream, c->fpart, nrb, n, g.vol, c->fpp, forces_dev);
  return hipGetLastError();
}

size_t ionic_force_partials(const arche_ctx* c) {
  int rpb = 0;
  return (size_t)force_row_blocks(c, &rpb) * c->n_atoms * 3;
}

// spectral part of P_ie (host out)
hipError_t ionic_pressure_ie(arche_ctx* c, const cplx* nhat, double* out) {
  const GridInfo& g = c->g;
  const int nbh = red_blocks(g.nh);
  hipLaunchKernelGGL(k_pressure_ie, dim3(nbh), dim3(ARCHE_BLOCK), 0, c->stream, nhat, c->Sp, c->Sm, c->sp, g,
                     c->partials);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(c->partials, nbh, 1, c->sums, c->stream));
  HIP_TRY(hipMemcpyAsync(out, c->sums, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return hipStreamSynchronize(c->stream);
}

// shell index of every half-box point: |m|^2 for cubic cells, (mx^2, my^2, mz^2) otherwise
hipError_t ionic_shells(arche_ctx* c) {
  const GridInfo& g = c->g;
  const bool cubic = g.N[0] == g.N[1] && g.N[1] == g.N[2] && g.L[0] == g.L[1] && g.L[1] == g.L[2];
  const int64_t P = (int64_t)std::max(g.N[0], std::max(g.N[1], g.N[2])) * std::max(g.N[0], std::max(g.N[1], g.N[2])) / 4 + 1;
  std::vector<int64_t> key(g.nh);
  for (int64_t m = 0; m < g.nh; ++m) {
    const int iz = (int)(m % g.Nh);
    const int64_t r = m / g.Nh;
    const int iy = (int)(r % g.N[1]);
    const int ix = (int)(r / g.N[1]);
    const int64_t mx = ix <= g.N[0] / 2 ? ix : ix - g.N[0];
    const int64_t my = iy <= g.N[1] / 2 ? iy : iy - g.N[1];
    const int64_t mz = iz;
    key[m] = cubic ? mx * mx + my * my + mz * mz : (mx * mx * P + my * my) * P + mz * mz;
  }
  std::vector<int32_t> perm(g.nh);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  std::vector<int32_t> shell_of(g.nh), off;
  int ns = 0;
  for (int64_t q = 0; q < g.nh; ++q) {
    if (q == 0 || key[perm[q]] != key[perm[q - 1]]) {
      off.push_back((int32_t)q);
      ++ns;
    }
    shell_of[perm[q]] = ns - 1;
  }
  off.push_back((int32_t)g.nh);
  c->nshell = ns;
  if (c->dalloc_.get((void**)&c->shell_of, g.nh * sizeof(int32_t), c->stream) != hipSuccess) return hipErrorOutOfMemory;
  if (c->dalloc_.get((void**)&c->shell_perm, g.nh * sizeof(int32_t), c->stream) != hipSuccess) return hipErrorOutOfMemory;
  if (c->dalloc_.get((void**)&c->shell_off, (ns + 1) * sizeof(int32_t), c->stream) != hipSuccess) return hipErrorOutOfMemory;
  if (c->dalloc_.get((void**)&c->shell_g, ns * sizeof(double), c->stream) != hipSuccess) return hipErrorOutOfMemory;
  HIP_TRY(hipMemcpy(c->shell_of, shell_of.data(), g.nh * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->shell_perm, perm.data(), g.nh * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->shell_off, off.data(), (ns + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  return hipSuccess;
}

// Floor n at GUESS_FLOOR n_0 and rescale it to N_e electrons; *ok = false (n
// left floored, not rescaled) when the floor added more than MAX_FLOOR_CHARGE
// of the charge or the result is not finite.  A guess that rings negative over
// a region is rejected: floored plateaus make the von Weizsaecker potential
// nearly singular and the SCF diverges; the few points a rounding-level ring
// touches are floored at 1e-3 n_0 rather than near zero for the same reason.
constexpr double GUESS_FLOOR = 1e-3;
constexpr double MAX_FLOOR_CHARGE = 1e-6;
hipError_t scf_floor_renorm(arche_ctx* c, double* n, bool* ok) {
  const GridInfo& g = c->g;
  const double n0 = c->Ne / g.vol;
  const int nb = red_blocks(g.ng);
  hipLaunchKernelGGL(k_floor, dim3(nb), dim3(ARCHE_BLOCK), 0, c->stream, n, g.ng, GUESS_FLOOR * n0, c->partials);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(c->partials, nb, 1, c->sums, c->stream));
  HIP_TRY(finish_sums(c->partials + nb, nb, 1, c->sums + 1, c->stream));
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, c->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double raw = g.dv * h[0], fl = g.dv * h[1];
  *ok = std::fabs(fl - raw) <= MAX_FLOOR_CHARGE * c->Ne && fl > 0.0 && std::isfinite(fl);
  if (!*ok) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, n, g.ng, c->Ne / fl);
  return hipGetLastError();
}

// n_i = the one-center guess (Sec. 2.5.1) from the previous converged step
// (g per shell, n^_i = g (SZ+ + SZ-)/2 at the new positions, C2R), floored and
// rescaled; uniform when scf_floor_renorm rejects it.  No derived fields.
hipError_t scf_one_center_density(arche_ctx* c, int* used_fallback, double* raw, double* delta) {
  const GridInfo& g = c->g;
  *used_fallback = 0;
  hipLaunchKernelGGL(k_shell_profile, dim3((c->nshell + ARCHE_BLOCK / 64 - 1) / (ARCHE_BLOCK / 64)), dim3(ARCHE_BLOCK), 0,
                     c->stream, c->prev_nhat, c->prev_SZp, c->prev_SZm, c->shell_perm, c->shell_off, c->nshell, g,
                     c->sumZ2, c->shell_g);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_one_center_hat, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->shell_g,
                     c->shell_of, c->SZp, c->SZm, g, c->ctmp);
  HIP_TRY(hipGetLastError());
  if (delta) {
    // the superposition's change: g^ (SZ_new - SZ_prev), into delta (via ctmp2)
    hipLaunchKernelGGL(k_one_center_hat, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->shell_g,
                       c->shell_of, c->prev_SZp, c->prev_SZm, g, c->ctmp2);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_spec_sub, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->ctmp, c->ctmp2, g.nh);
    HIP_TRY(hipGetLastError());
    HIP_TRY(fft_c2r(&c->plan, c->ctmp2, delta, 1.0 / g.vol, c->stream));
  }
  HIP_TRY(fft_c2r(&c->plan, c->ctmp, c->n_i, 1.0 / g.vol, c->stream));
  if (raw) HIP_TRY(hipMemcpyAsync(raw, c->n_i, g.ng * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  bool ok = false;
  HIP_TRY(scf_floor_renorm(c, c->n_i, &ok));
  if (!ok) {
    *used_fallback = 1;
    hipLaunchKernelGGL(k_fill_ni, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, c->n_i, g.ng, c->Ne / g.vol);
    HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

// s^ <- s^ exp(-(|k|/kc)^2) on the half spectrum
__global__ void __launch_bounds__(ARCHE_BLOCK) k_spec_gauss(cplx* s, GridInfo g, double kc) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    const int iz = (int)(m % g.Nh);
    const int64_t rr = m / g.Nh;
    const int iy = (int)(rr % g.N[1]), ix = (int)(rr / g.N[1]);
    const double kx = (double)(ix <= g.N[0] / 2 ? ix : ix - g.N[0]) / g.L[0];
    const double ky = (double)(iy <= g.N[1] / 2 ? iy : iy - g.N[1]) / g.L[1];
    const double kz = (double)iz / g.L[2];
    s[m] = cscale(s[m], exp(-(kx * kx + ky * ky + kz * kz) / (kc * kc)));
  }
}
// n = max(p + n0 r, 0.1 p)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_learned_combine(const double* p, const double* r, double n0, double* n, int64_t ng) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (int64_t)gridDim.x * blockDim.x) {
    const double rp = r[i], pp = p[i];
    n[i] = rp == rp ? fmax(pp + n0 * rp, 0.1 * pp) : rp;
  }
}

__global__ void __launch_bounds__(ARCHE_BLOCK) k_add_scalar(double* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] += v;
}
hipError_t scf_add_scalar(arche_ctx* c, double* x, double v) {
  hipLaunchKernelGGL(k_add_scalar, dim3(grid_for(c->g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, x, c->g.ng, v);
  return hipGetLastError();
}

// The learned proposal from the network's output r (in rtmp): r is low-passed
// with exp(-(|k|/kc)^2), kc a quarter of the smallest Nyquist frequency (the
// SCF converges slowly from guesses with short-wavelength error, which the
// network's output carries), then n = max(p + n0 r, 0.1 p) -> rtmp.
hipError_t scf_learned_proposal(arche_ctx* c) {
  const GridInfo& g = c->g;
  double kc = 1e300;
  for (int a = 0; a < 3; ++a) kc = std::min(kc, 0.25 * 0.5 * g.N[a] / g.L[a]);
  HIP_TRY(fft_r2c(&c->plan, c->rtmp, c->ctmp, 1.0, g.dv, c->stream));
  hipLaunchKernelGGL(k_spec_gauss, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->ctmp, g, kc);
  HIP_TRY(hipGetLastError());
  HIP_TRY(fft_c2r(&c->plan, c->ctmp, c->lap_a, 1.0 / g.vol, c->stream));
  hipLaunchKernelGGL(k_learned_combine, dim3(grid_for(g.ng)), dim3(ARCHE_BLOCK), 0, c->stream, c->n_a, c->lap_a,
                     c->Ne / g.vol, c->rtmp, g.ng);
  return hipGetLastError();
}

hipError_t scf_initial_one_center(arche_ctx* c, int* used_fallback) {
  HIP_TRY(scf_one_center_density(c, used_fallback, nullptr, nullptr));
  return scf_prepare_input(c);
}

// Reciprocal-space and pair sums of the stress tensor at the converged state
// (see k_stress_recip): out24 = ee[6], vw[6], ie[6], pm[6]; pp6 = the pair
// tensor summed over atoms.  shat may be null (no von Weizsaecker term).
hipError_t ionic_stress_sums(arche_ctx* c, const cplx* nhat, const cplx* shat, double alpha, double* out24,
                             double* pp6) {
  const GridInfo& g = c->g;
  const int nbh = red_blocks(g.nh);
  const int n = c->n_atoms;
  double* pp = c->partials;
  double* part = c->partials + 6 * (size_t)n;
  hipLaunchKernelGGL(k_ewald_pair_stress, dim3(n), dim3(ARCHE_BLOCK), 0,
                     c->stream, c->pos, c->Zatom, n, g, alpha, pp);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(pp, n, 6, c->sums, c->stream));
  hipLaunchKernelGGL(k_stress_recip, dim3(nbh), dim3(ARCHE_BLOCK), 0, c->stream, nhat, shat, c->Sp, c->Sm, c->SZp,
                     c->SZm, c->sp, g, alpha, part);
  HIP_TRY(hipGetLastError());
  HIP_TRY(finish_sums(part, nbh, 24, c->sums + 6, c->stream));
  double h[30];
  HIP_TRY(hipMemcpyAsync(h, c->sums, 30 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int q = 0; q < 6; ++q) pp6[q] = h[q];
  for (int q = 0; q < 24; ++q) out24[q] = h[6 + q];
  return hipSuccess;
}
