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

// phase tables exp(-2 pi i k_m x / L) for atom j and box index m (axis a), z only m <= Nz/2
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_phases(const double* pos, int n_atoms, GridInfo g, cplx* phx, cplx* phy, cplx* phz) {
  const int64_t total = (int64_t)n_atoms * (g.N[0] + g.N[1] + g.Nh);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = q / (g.N[0] + g.N[1] + g.Nh);
    int r = (int)(q - j * (g.N[0] + g.N[1] + g.Nh));
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
    const int m = axis == 2 ? i : box_m(i, g.N[axis]);
    double f = pos[j * 3 + axis] / g.L[axis];
    f -= floor(f);
    double th = (double)m * f;
    th -= rint(th);  // exp(-2 pi i th) is 1-periodic in th
    double s, c;
    sincospi(2.0 * th, &s, &c);
    cplx v{c, -s};
    if (axis == 0)
      phx[j * g.N[0] + i] = v;
    else if (axis == 1)
      phy[j * g.N[1] + i] = v;
    else
      phz[j * g.Nh + i] = v;
  }
}

// S+_s(m) = sum_{j in s} P_j(k_m), S-_s(m) = sum_{j in s} P_j(k~_m), atoms sorted by species
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_structure(const cplx* __restrict__ phx, const cplx* __restrict__ phy, const cplx* __restrict__ phz,
            const int* __restrict__ order, const int* __restrict__ sp_begin, int ns, GridInfo g, cplx* Sp, cplx* Sm) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < g.nh; m += (int64_t)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    const bool nx = 2 * ix == g.N[0], ny = 2 * iy == g.N[1], nz = 2 * iz == g.N[2];
    const bool nyq = nx || ny || nz;
    for (int s = 0; s < ns; ++s) {
      cplx ap{0.0, 0.0}, am{0.0, 0.0};
      for (int q = sp_begin[s]; q < sp_begin[s + 1]; ++q) {
        const int j = order[q];
        cplx a{1.0, 0.0}, b{1.0, 0.0};
        const cplx px = phx[(int64_t)j * g.N[0] + ix];
        const cplx py = phy[(int64_t)j * g.N[1] + iy];
        const cplx pz = phz[(int64_t)j * g.Nh + iz];
        if (nx) b = px; else a = px;
        if (ny) b = cmul(b, py); else a = cmul(a, py);
        if (nz) b = cmul(b, pz); else a = cmul(a, pz);
        ap = cadd(ap, cmul(a, b));
        if (nyq) am = cadd(am, cmul(a, cconj(b)));
      }
      Sp[(int64_t)s * g.nh + m] = ap;
      Sm[(int64_t)s * g.nh + m] = nyq ? am : ap;
    }
  }
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

// Ewald real-space pairs (minimum image): per-atom forces and half the pair energy
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_ewald_pairs(const double* pos, const double* Zat, int n, GridInfo g, double alpha, double* F, double* Uj) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double xj = pos[3 * j], yj = pos[3 * j + 1], zj = pos[3 * j + 2];
  double fx = 0, fy = 0, fz = 0, u = 0;
  const double c2 = 2.0 * alpha / sqrt(PI);
  for (int l = 0; l < n; ++l) {
    if (l == j) continue;
    double d[3] = {xj - pos[3 * l], yj - pos[3 * l + 1], zj - pos[3 * l + 2]};
    for (int a = 0; a < 3; ++a) d[a] -= g.L[a] * rint(d[a] / g.L[a]);
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = sqrt(r2);
    const double zz = Zat[j] * Zat[l];
    const double e = erfc(alpha * r) / r;
    u += 0.5 * zz * e;
    const double coef = zz * (e + c2 * exp(-alpha * alpha * r2)) / r2;
    fx += coef * d[0];
    fy += coef * d[1];
    fz += coef * d[2];
  }
  F[3 * j] = fx;
  F[3 * j + 1] = fy;
  F[3 * j + 2] = fz;
  Uj[j] = u;
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

// F_j = -(2 pi/|Omega|) sum over the full box of Im(W(k) exp(-2 pi i k.r_j)) k, as
// partial sums over chunks of the half box for a tile of ATILE atoms.
constexpr int ATILE = 8;
constexpr int MCHUNK = ARCHE_BLOCK * 16;

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_force_contract(const cplx* __restrict__ Wp, const cplx* __restrict__ Wm, const cplx* __restrict__ phx,
                 const cplx* __restrict__ phy, const cplx* __restrict__ phz, const int* __restrict__ spec, int n_atoms,
                 GridInfo g, double* part /*[nchunk][n_atoms][3]*/) {
  __shared__ double sh[ARCHE_BLOCK / 64];
  const int tile = blockIdx.y;
  const int chunk = blockIdx.x;
  const int j0 = tile * ATILE;
  const int nj = min(ATILE, n_atoms - j0);
  double acc[ATILE][3];
  for (int t = 0; t < ATILE; ++t) acc[t][0] = acc[t][1] = acc[t][2] = 0.0;
  const int64_t mend = min((int64_t)(chunk + 1) * MCHUNK, g.nh);
  for (int64_t m = (int64_t)chunk * MCHUNK + threadIdx.x; m < mend; m += blockDim.x) {
    int ix, iy, iz;
    half_index(m, g.N[1], g.Nh, ix, iy, iz);
    double k[3];
    kvec(ix, iy, iz, g, k);
    const bool nx = 2 * ix == g.N[0], ny = 2 * iy == g.N[1];
    const bool interior = iz != 0 && 2 * iz != g.N[2];
    const bool mirror_differs = interior && (nx || ny);
    const double wgt = (interior && !mirror_differs) ? 2.0 : 1.0;
    const double kt[3] = {nx ? -k[0] : k[0], ny ? -k[1] : k[1], k[2]};
#pragma unroll
    for (int t = 0; t < ATILE; ++t) {
      if (t >= nj) break;
      const int j = j0 + t;
      const int s = spec[j];
      const cplx px = phx[(int64_t)j * g.N[0] + ix];
      const cplx py = phy[(int64_t)j * g.N[1] + iy];
      const cplx pz = phz[(int64_t)j * g.Nh + iz];
      const cplx wp = Wp[(int64_t)s * g.nh + m];
      const cplx P = cmul(cmul(px, py), pz);
      const double im = wgt * (wp.x * P.y + wp.y * P.x);
      acc[t][0] += im * k[0];
      acc[t][1] += im * k[1];
      acc[t][2] += im * k[2];
      if (mirror_differs) {
        const cplx wm = Wm[(int64_t)s * g.nh + m];
        const cplx Pt = cmul(cmul(nx ? cconj(px) : px, ny ? cconj(py) : py), pz);
        const double im2 = wm.x * Pt.y + wm.y * Pt.x;
        acc[t][0] += im2 * kt[0];
        acc[t][1] += im2 * kt[1];
        acc[t][2] += im2 * kt[2];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < ATILE; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double v = block_sum(acc[t][a], sh);
      if (threadIdx.x == 0 && t < nj) part[((int64_t)chunk * n_atoms + j0 + t) * 3 + a] = v;
    }
}

// F_j = -(2 pi/|Omega|) sum_chunks part + F^pp_j, in fixed chunk order
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_force_finish(const double* part, int nchunk, int n_atoms, double vol, const double* Fpp, double* F) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_atoms * 3) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * n_atoms * 3 + q];
  F[q] = -2.0 * PI / vol * s + Fpp[q];
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

// one-center profile per shell: g = sum Re(n^ conj SZ) / sum |SZ|^2 over the full box
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_shell_profile(const cplx* nhat, const cplx* SZp, const cplx* SZm, const int* perm, const int* off, int nshell,
                GridInfo g, double sumZ2, double* gsh) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshell) return;
  double num = 0.0, den = 0.0, cnt = 0.0;
  for (int q = off[s]; q < off[s + 1]; ++q) {
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
  gsh[s] = den > SHELL_CUT * cnt * sumZ2 ? num / den : 0.0;
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
// six components per atom [j][6]
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_ewald_pair_stress(const double* pos, const double* Zat, int n, GridInfo g, double alpha, double* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double xj = pos[3 * j], yj = pos[3 * j + 1], zj = pos[3 * j + 2];
  const double c2 = 2.0 * alpha / sqrt(PI);
  double o[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 0; l < n; ++l) {
    if (l == j) continue;
    double d[3] = {xj - pos[3 * l], yj - pos[3 * l + 1], zj - pos[3 * l + 2]};
    for (int a = 0; a < 3; ++a) d[a] -= g.L[a] * rint(d[a] / g.L[a]);
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = sqrt(r2);
    const double coef = 0.5 * Zat[j] * Zat[l] * (erfc(alpha * r) / r + c2 * exp(-alpha * alpha * r2)) / r2;
    kk6(d, coef, o);
  }
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
                     c->stream, c->pos, c->n_atoms, g, c->phx, c->phy, c->phz);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_structure, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, c->phx, c->phy, c->phz,
                     c->sp_order, c->sp_begin, c->n_species, g, c->Sp, c->Sm);
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
  hipLaunchKernelGGL(k_ewald_pairs, dim3((n + ARCHE_BLOCK - 1) / ARCHE_BLOCK), dim3(ARCHE_BLOCK), 0, c->stream, c->pos,
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

// forces (device [n][3]) from the converged spectrum nhat; needs ionic_ewald first (F^pp)
hipError_t ionic_forces(arche_ctx* c, const cplx* nhat, double* forces_dev) {
  const GridInfo& g = c->g;
  const double alpha = ewald_alpha(c);
  hipLaunchKernelGGL(k_force_weights, dim3(grid_for(g.nh)), dim3(ARCHE_BLOCK), 0, c->stream, nhat, c->SZp, c->SZm,
                     c->sp, g, alpha, c->Wp, c->Wm);
  HIP_TRY(hipGetLastError());
  const int nchunk = (int)((g.nh + MCHUNK - 1) / MCHUNK);
  const int ntile = (c->n_atoms + ATILE - 1) / ATILE;
  hipLaunchKernelGGL(k_force_contract, dim3(nchunk, ntile), dim3(ARCHE_BLOCK), 0, c->stream, c->Wp, c->Wm, c->phx,
                     c->phy, c->phz, c->spec_d, c->n_atoms, g, c->fpart);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_force_finish, dim3((3 * c->n_atoms + ARCHE_BLOCK - 1) / ARCHE_BLOCK), dim3(ARCHE_BLOCK), 0,
                     c->stream, c->fpart, nchunk, c->n_atoms, g.vol, c->fpp, forces_dev);
  return hipGetLastError();
}

size_t ionic_force_partials(const arche_ctx* c) {
  const int nchunk = (int)((c->g.nh + MCHUNK - 1) / MCHUNK);
  return (size_t)nchunk * c->n_atoms * 3;
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
  hipLaunchKernelGGL(k_shell_profile, dim3((c->nshell + ARCHE_BLOCK - 1) / ARCHE_BLOCK), dim3(ARCHE_BLOCK), 0,
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
  hipLaunchKernelGGL(k_ewald_pair_stress, dim3((n + ARCHE_BLOCK - 1) / ARCHE_BLOCK), dim3(ARCHE_BLOCK), 0,
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
