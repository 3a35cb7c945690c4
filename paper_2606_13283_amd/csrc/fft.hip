// FP64 3D real<->complex FFT for gfx950 (see fft.h for the layout and passes).
#include "fft.h"
#include "fft_bodies.h"
#include "profile.h"

#include <cmath>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <vector>

namespace {

using namespace fftct;

struct Radices {
  int nst;
  int r[8];
};

// multiply by (sign * i)
__device__ inline cplx mul_si(cplx z, double sign) { return cplx{-sign * z.y, sign * z.x}; }

__device__ inline void bfly2(cplx* v) {
  cplx a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ inline void bfly3(cplx* v, double sign) {
  const double H = 0.86602540378443864676;  // sqrt(3)/2
  cplx a = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
  cplx m = cplx{a.x - 0.5 * s.x, a.y - 0.5 * s.y};
  cplx t = mul_si(cscale(d, H), sign);
  v[0] = cadd(a, s);
  v[1] = cadd(m, t);
  v[2] = csub(m, t);
}

__device__ inline void bfly4(cplx* v, double sign) {
  cplx t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  cplx t2 = cadd(v[1], v[3]), t3 = mul_si(csub(v[1], v[3]), sign);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

__device__ inline void bfly5(cplx* v, double sign) {
  const double C1 = 0.30901699437494742410;   // cos(2 pi/5)
  const double C2 = -0.80901699437494742410;  // cos(4 pi/5)
  const double S1 = 0.95105651629515357212;   // sin(2 pi/5)
  const double S2 = 0.58778525229247312917;   // sin(4 pi/5)
  cplx a = v[0];
  cplx s1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
  cplx s2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
  cplx r1 = cplx{a.x + C1 * s1.x + C2 * s2.x, a.y + C1 * s1.y + C2 * s2.y};
  cplx r2 = cplx{a.x + C2 * s1.x + C1 * s2.x, a.y + C2 * s1.y + C1 * s2.y};
  cplx i1 = mul_si(cplx{S1 * d1.x + S2 * d2.x, S1 * d1.y + S2 * d2.y}, sign);
  cplx i2 = mul_si(cplx{S2 * d1.x - S1 * d2.x, S2 * d1.y - S1 * d2.y}, sign);
  v[0] = cadd(a, cadd(s1, s2));
  v[1] = cadd(r1, i1);
  v[4] = csub(r1, i1);
  v[2] = cadd(r2, i2);
  v[3] = csub(r2, i2);
}

template <int R>
__device__ inline void bfly(cplx* v, double sg) {
  if constexpr (R == 2) bfly2(v);
  else if constexpr (R == 3) bfly3(v, sg);
  else if constexpr (R == 4) bfly4(v, sg);
  else bfly5(v, sg);
}

// One radix-R Stockham stage over `nlines` lines (all indices compile-time
// unrolled in R, so the butterfly stays in registers).
template <int R>
__device__ inline void stockham_stage(const cplx* src, cplx* dst, const cplx* tw, int L, int nlines, int es,
                                      int ls, int Ns, int sign, bool line_fast) {
  const int nb = L / R;
  const int total = nb * nlines;
  const int tstep = L / (Ns * R);
  const double sg = (double)sign;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int line, j;
    if (line_fast) {
      line = t % nlines;
      j = t / nlines;
    } else {
      j = t % nb;
      line = t / nb;
    }
    const int k = j % Ns;
    cplx v[R];
    const cplx* in = src + line * ls;
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[(j + r * nb) * es];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cplx w = tw[r * k * tstep];
      if (sign > 0) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    bfly<R>(v, sg);
    const int base = (j / Ns) * Ns * R + k;
    cplx* out = dst + line * ls;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(base + r * Ns) * es] = v[r];
  }
}

// Mixed-radix Stockham transform of `nlines` lines of length L held in LDS.
// Element k of line b sits at buf[b*ls + k*es].  `line_fast` maps consecutive
// threads to consecutive lines (for line-interleaved tiles) instead of to
// consecutive butterflies of one line.  Returns the buffer holding the result.
__device__ cplx* lds_fft(cplx* src, cplx* dst, const cplx* tw, int L, int nlines, int es, int ls,
                         const Radices& rp, int sign, bool line_fast) {
  int Ns = 1;
  for (int s = 0; s < rp.nst; ++s) {
    const int R = rp.r[s];
    switch (R) {
      case 2: stockham_stage<2>(src, dst, tw, L, nlines, es, ls, Ns, sign, line_fast); break;
      case 3: stockham_stage<3>(src, dst, tw, L, nlines, es, ls, Ns, sign, line_fast); break;
      case 4: stockham_stage<4>(src, dst, tw, L, nlines, es, ls, Ns, sign, line_fast); break;
      default: stockham_stage<5>(src, dst, tw, L, nlines, es, ls, Ns, sign, line_fast); break;
    }
    __syncthreads();
    cplx* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= R;
  }
  return src;
}

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_fft_z_r2c(const double* __restrict__ in, cplx* __restrict__ out, const cplx* __restrict__ tw_g,
            int Nz, int Nh, int64_t npairs, int B, Radices rp, double in_scale, double out_scale) {
  extern __shared__ cplx sm[];
  const int pitch = Nz + 2;
  cplx* a = sm;
  cplx* b = sm + B * pitch;
  cplx* tw = sm + 2 * B * pitch;
  for (int i = threadIdx.x; i < Nz; i += blockDim.x) tw[i] = tw_g[i];
  const int64_t p0 = (int64_t)blockIdx.x * B;
  const int nb = (int)((npairs - p0) < B ? (npairs - p0) : B);
  const double* src = in + p0 * 2 * Nz;
  for (int q = threadIdx.x; q < nb * 2 * Nz; q += blockDim.x) {
    int l = q / (2 * Nz);
    int w = q - l * 2 * Nz;
    int r = w / Nz;
    int k = w - r * Nz;
    double v = src[q] * in_scale;
    if (r == 0)
      a[l * pitch + k].x = v;
    else
      a[l * pitch + k].y = v;
  }
  __syncthreads();
  cplx* res = lds_fft(a, b, tw, Nz, nb, 1, pitch, rp, -1, false);
  cplx* dst = out + p0 * 2 * Nh;
  for (int q = threadIdx.x; q < nb * 2 * Nh; q += blockDim.x) {
    int l = q / (2 * Nh);
    int w = q - l * 2 * Nh;
    int r = w / Nh;
    int k = w - r * Nh;
    cplx zk = res[l * pitch + k];
    cplx zn = res[l * pitch + (k == 0 ? 0 : Nz - k)];
    cplx v;
    if (r == 0)
      v = cplx{0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y)};
    else
      v = cplx{0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x)};
    dst[q] = cscale(v, out_scale);
  }
}

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_fft_z_c2r(const cplx* __restrict__ in, double* __restrict__ out, const cplx* __restrict__ tw_g,
            int Nz, int Nh, int64_t npairs, int B, Radices rp, double out_scale) {
  extern __shared__ cplx sm[];
  const int pitch = Nz + 2;
  cplx* a = sm;
  cplx* b = sm + B * pitch;
  cplx* tw = sm + 2 * B * pitch;
  for (int i = threadIdx.x; i < Nz; i += blockDim.x) tw[i] = tw_g[i];
  const int64_t p0 = (int64_t)blockIdx.x * B;
  const int nb = (int)((npairs - p0) < B ? (npairs - p0) : B);
  const cplx* src = in + p0 * 2 * Nh;
  // stage the two half rows of each pair (2*Nh <= pitch values) contiguously
  for (int q = threadIdx.x; q < nb * 2 * Nh; q += blockDim.x) {
    int l = q / (2 * Nh);
    int w = q - l * 2 * Nh;
    b[l * pitch + w] = src[q];
  }
  __syncthreads();
  const int half = Nz / 2;
  for (int q = threadIdx.x; q < nb * Nz; q += blockDim.x) {
    int l = q / Nz;
    int k = q - l * Nz;
    const cplx* X = b + l * pitch;
    const cplx* Y = X + Nh;
    cplx x, y;
    if (k == 0 || k == half) {
      x = cplx{X[k].x, 0.0};
      y = cplx{Y[k].x, 0.0};
    } else if (k < half) {
      x = X[k];
      y = Y[k];
    } else {
      x = cconj(X[Nz - k]);
      y = cconj(Y[Nz - k]);
    }
    a[l * pitch + k] = cplx{x.x - y.y, x.y + y.x};
  }
  __syncthreads();
  cplx* res = lds_fft(a, b, tw, Nz, nb, 1, pitch, rp, +1, false);
  double* dst = out + p0 * 2 * Nz;
  for (int q = threadIdx.x; q < nb * 2 * Nz; q += blockDim.x) {
    int l = q / (2 * Nz);
    int w = q - l * 2 * Nz;
    int r = w / Nz;
    int k = w - r * Nz;
    cplx z = res[l * pitch + k];
    dst[q] = (r == 0 ? z.x : z.y) * out_scale;
  }
}

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_fft_strided(cplx* __restrict__ data, const cplx* __restrict__ tw_g, int L, int64_t es, int64_t os,
              int ncols, int TK, int nchunk, Radices rp, int sign, double scale) {
  extern __shared__ cplx sm[];
  cplx* a = sm;
  cplx* b = sm + L * TK;
  cplx* tw = sm + 2 * L * TK;
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = tw_g[i];
  const int o = blockIdx.x / nchunk;
  const int c0 = (blockIdx.x - o * nchunk) * TK;
  const int nc = (ncols - c0) < TK ? (ncols - c0) : TK;
  cplx* base = data + (int64_t)o * os + c0;
  for (int q = threadIdx.x; q < L * TK; q += blockDim.x) {
    int k = q / TK;
    int c = q - k * TK;
    a[q] = (c < nc) ? base[(int64_t)k * es + c] : cplx{0.0, 0.0};
  }
  __syncthreads();
  cplx* res = lds_fft(a, b, tw, L, TK, TK, 1, rp, sign, true);
  for (int q = threadIdx.x; q < L * TK; q += blockDim.x) {
    int k = q / TK;
    int c = q - k * TK;
    if (c < nc) base[(int64_t)k * es + c] = cscale(res[q], scale);
  }
}

// ---------------------------------------------------------------------------
// Compile-time kernels (fft_plans.h, tile bodies in fft_bodies.h) for the
// supported line lengths.  A pass whose FftFuse names a stop flag does nothing
// once it is set (a converged SCF).
__device__ inline bool fft_stopped(const FftFuse& f) { return f.stop && *f.stop; }

template <int L, int TK, int S, int MODE, int NT>
__global__ void __launch_bounds__(NT) k_strided_ct(StridedArgs A) {
  if (fft_stopped(A.f)) return;
  __shared__ cplx lds[strided_lds<L, TK>()];
  __shared__ cplx tw[L];
  __shared__ double sh[NT / 64];
  strided_body<L, TK, S, MODE, NT>(A, blockIdx.x, lds, tw, sh);
}

template <int L, int B, int FIN, int NT>
__global__ void __launch_bounds__(NT) k_z_r2c_ct(ZArgs A) {
  if (fft_stopped(A.f)) return;
  __shared__ cplx lds[z_r2c_lds<L, B>()];
  __shared__ cplx tw[L];
  z_r2c_body<L, B, FIN, NT>(A, blockIdx.x, lds, tw);
}

template <int L, int B, int FOUT, int NT>
__global__ void __launch_bounds__(NT) k_z_c2r_ct(ZArgs A) {
  if (fft_stopped(A.f)) return;
  __shared__ cplx lds[z_c2r_lds<L, B>()];
  __shared__ cplx tw[L];
  __shared__ double sh[NT / 64];
  z_c2r_body<L, B, FOUT, NT>(A, blockIdx.x, lds, tw, sh);
}

// Plane passes (N_y = N_z = L): one block of PLANE_NT threads per x plane.
constexpr int PLANE_NT = 1024;
template <int L, int FIN>
__global__ void __launch_bounds__(PLANE_NT) k_zy_r2c(ZArgs A) {
  if (fft_stopped(A.f)) return;
  __shared__ cplx plane[plane_lds<L>()];
  __shared__ cplx tw[L];
  zy_r2c_body<L, FIN, PLANE_NT>(A, blockIdx.x, plane, tw);
}
template <int L, int FOUT>
__global__ void __launch_bounds__(PLANE_NT) k_yz_c2r(ZArgs A) {
  if (fft_stopped(A.f)) return;
  __shared__ cplx plane[plane_lds<L>()];
  __shared__ cplx tw[L];
  __shared__ double sh[PLANE_NT / 64];
  yz_c2r_body<L, FOUT, PLANE_NT>(A, blockIdx.x, plane, tw, sh);
}
#define ARCHE_PLANE_SIZES(X) X(128)
bool plane_supported(int L) {
  switch (L) {
#define X(n) case n:
    ARCHE_PLANE_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}
template <int L>
hipError_t launch_plane_L(const FftPass& ps, hipStream_t s) {
  const dim3 grid(ps.nblocks), blk(PLANE_NT);
  if (ps.kind == FFT_PASS_ZY_R2C) {
    if (ps.mode == 0) hipLaunchKernelGGL((k_zy_r2c<L, 0>), grid, blk, 0, s, ps.z);
    else if (ps.mode == 1) hipLaunchKernelGGL((k_zy_r2c<L, 1>), grid, blk, 0, s, ps.z);
    else hipLaunchKernelGGL((k_zy_r2c<L, 2>), grid, blk, 0, s, ps.z);
  } else {
    if (ps.mode == 0) hipLaunchKernelGGL((k_yz_c2r<L, 0>), grid, blk, 0, s, ps.z);
    else hipLaunchKernelGGL((k_yz_c2r<L, 1>), grid, blk, 0, s, ps.z);
  }
  return hipGetLastError();
}
hipError_t launch_plane(const FftPass& ps, hipStream_t s) {
  switch (ps.L) {
#define X(n) \
  case n:    \
    return launch_plane_L<n>(ps, s);
    ARCHE_PLANE_SIZES(X)
#undef X
    default:
      return hipErrorNotSupported;
  }
}

// Two independent plane passes in one launch: blocks [0, n1) run the first
// (direction K1: 0 R2C z+y, 1 C2R y+z; mode M1), the rest the second, so the
// pair fills the CUs that one pass over Nx planes leaves idle.
template <int L, int K, int M>
__device__ inline void plane_body(const ZArgs& A, unsigned bid, cplx* plane, cplx* tw, double* sh) {
  if constexpr (K == 0)
    zy_r2c_body<L, M, PLANE_NT>(A, bid, plane, tw);
  else
    yz_c2r_body<L, M, PLANE_NT>(A, bid, plane, tw, sh);
}
template <int L, int K1, int M1, int K2, int M2>
__global__ void __launch_bounds__(PLANE_NT) k_plane_dual(ZArgs A, ZArgs B, unsigned n1) {
  __shared__ cplx plane[plane_lds<L>()];
  __shared__ cplx tw[L];
  __shared__ double sh[PLANE_NT / 64];
  if (blockIdx.x < n1) {
    if (fft_stopped(A.f)) return;
    plane_body<L, K1, M1>(A, blockIdx.x, plane, tw, sh);
  } else {
    if (fft_stopped(B.f)) return;
    plane_body<L, K2, M2>(B, blockIdx.x - n1, plane, tw, sh);
  }
}
// An x pass and a plane pass in one launch: the Hartree C2R's x pass (spectral
// mixing on load) beside R2C(sqrt n_o)'s plane pass, both waiting only on the
// mixing weight.  The x pass runs in tiles of TKX = N_h columns (one k_y row of
// the (k_y, k_z) plane) with PLANE_NT threads, so that its N_y blocks take the
// CUs the N_x plane blocks leave free, each block holding one tile in LDS.
template <int L, int TKX, int SX, int MX, int K2, int M2>
__global__ void __launch_bounds__(PLANE_NT) k_xplane_dual(StridedArgs A, ZArgs B, unsigned n1) {
  constexpr int NE = plane_lds<L>() > strided_lds<L, TKX>() ? plane_lds<L>() : strided_lds<L, TKX>();
  __shared__ cplx lds[NE];
  __shared__ cplx tw[L];
  __shared__ double sh[PLANE_NT / 64];
  if (blockIdx.x < n1) {
    if (fft_stopped(A.f)) return;
    strided_body<L, TKX, SX, MX, PLANE_NT>(A, blockIdx.x, lds, tw, sh);
  } else {
    if (fft_stopped(B.f)) return;
    plane_body<L, K2, M2>(B, blockIdx.x - n1, lds, tw, sh);
  }
}
// Tile variants (autotuned per line length, fft.h): strided passes take TK
// columns per block with NT threads, z passes B row pairs with NT threads.
// Variant 0 is the default; line lengths of the batched set use only it.
constexpr int kStridedTK[3] = {CT_TK, 8, 4};
constexpr int kStridedNT[3] = {ARCHE_BLOCK, 128, 64};
template <int L>
constexpr bool tunable() {
  return L > 96;
}
template <int L>
constexpr int z_rows_var(int v) {
  return v == 0 ? ct_rows<L>() : (v == 1 ? 8 : 4);
}
constexpr int kZNT[3] = {ARCHE_BLOCK, 128, 64};

// line lengths with plane passes (and the x round trip of MODE 4)
template <int L>
constexpr bool plane_len() {
  return L == 128;
}
template <int L, int TK, int NT>
hipError_t launch_strided_tile(const FftPass& ps, hipStream_t s) {
  const dim3 grid(ps.nblocks), blk(NT);
  if (ps.mode == 0 && ps.sign < 0) hipLaunchKernelGGL((k_strided_ct<L, TK, -1, 0, NT>), grid, blk, 0, s, ps.s);
  else if (ps.mode == 0) hipLaunchKernelGGL((k_strided_ct<L, TK, +1, 0, NT>), grid, blk, 0, s, ps.s);
  else if (ps.mode == 1) hipLaunchKernelGGL((k_strided_ct<L, TK, -1, 1, NT>), grid, blk, 0, s, ps.s);
  else if (ps.mode == 2) hipLaunchKernelGGL((k_strided_ct<L, TK, -1, 2, NT>), grid, blk, 0, s, ps.s);
  else if (ps.mode == 3) hipLaunchKernelGGL((k_strided_ct<L, TK, +1, 3, NT>), grid, blk, 0, s, ps.s);
  else if constexpr (plane_len<L>()) hipLaunchKernelGGL((k_strided_ct<L, TK, -1, 4, NT>), grid, blk, 0, s, ps.s);
  else return hipErrorNotSupported;
  return hipGetLastError();
}
template <int L, int B, int NT>
hipError_t launch_z_tile(const FftPass& ps, hipStream_t s) {
  const dim3 grid(ps.nblocks), blk(NT);
  if (ps.kind == FFT_PASS_Z_R2C) {
    if (ps.mode == 0) hipLaunchKernelGGL((k_z_r2c_ct<L, B, 0, NT>), grid, blk, 0, s, ps.z);
    else if (ps.mode == 1) hipLaunchKernelGGL((k_z_r2c_ct<L, B, 1, NT>), grid, blk, 0, s, ps.z);
    else hipLaunchKernelGGL((k_z_r2c_ct<L, B, 2, NT>), grid, blk, 0, s, ps.z);
  } else {
    if (ps.mode == 0) hipLaunchKernelGGL((k_z_c2r_ct<L, B, 0, NT>), grid, blk, 0, s, ps.z);
    else hipLaunchKernelGGL((k_z_c2r_ct<L, B, 1, NT>), grid, blk, 0, s, ps.z);
  }
  return hipGetLastError();
}

template <int L>
hipError_t launch_pass(const FftPass& ps, hipStream_t s) {
  if (ps.kind == FFT_PASS_STRIDED) {
    if constexpr (tunable<L>()) {
      if (ps.var == 1) return launch_strided_tile<L, kStridedTK[1], kStridedNT[1]>(ps, s);
      if (ps.var == 2) return launch_strided_tile<L, kStridedTK[2], kStridedNT[2]>(ps, s);
    }
    return launch_strided_tile<L, kStridedTK[0], kStridedNT[0]>(ps, s);
  }
  if constexpr (tunable<L>()) {
    if (ps.var == 1) return launch_z_tile<L, z_rows_var<L>(1), kZNT[1]>(ps, s);
    if (ps.var == 2) return launch_z_tile<L, z_rows_var<L>(2), kZNT[2]>(ps, s);
  }
  return launch_z_tile<L, z_rows_var<L>(0), kZNT[0]>(ps, s);
}
template <int L>
constexpr int z_rows() {
  return ct_rows<L>();
}

// kind 0: strided, 1: z r2c, 2: z c2r.  Returns hipErrorNotSupported for other sizes.
#define ARCHE_CT_SIZES(X) \
  X(16) X(20) X(24) X(30) X(32) X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(80) X(96) X(100) X(120) X(128) X(144) \
  X(160) X(180) X(192) X(256)

bool ct_supported(int L) {
  switch (L) {
#define X(n) case n:
    ARCHE_CT_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

// direction code of a plane pass (0 R2C, 1 C2R), -1 otherwise
int plane_dir(const FftPass& p) {
  return p.kind == FFT_PASS_ZY_R2C ? 0 : (p.kind == FFT_PASS_YZ_C2R ? 1 : -1);
}

// The pairs the SCF iteration launches together: the plane passes of R2C(n_a)
// and R2C(sqrt n_a); where the x length has the round trip, the U_H x pass with
// the U_vW plane pass, the Hartree C2R's x pass with R2C(sqrt n_o)'s plane pass,
// and the Hartree C2R's plane pass with that of the C2R back from the
// Laplacian (elsewhere, with R2C(sqrt n_o)'s plane pass).
template <int L>
bool launch_dual_L(const FftPass& a, const FftPass& b, hipStream_t s, hipError_t* e) {
  const dim3 blk_p(PLANE_NT);
  const int da = plane_dir(a), db = plane_dir(b);
  if (da == 1 && a.mode == 0 && db == 1 && b.mode == 0) {
    hipLaunchKernelGGL((k_plane_dual<L, 1, 0, 1, 0>), dim3(a.nblocks + b.nblocks), blk_p, 0, s, a.z, b.z, a.nblocks);
  } else if (a.kind == FFT_PASS_STRIDED && a.sign < 0 && a.mode == 2 && db == 1 && b.mode == 1) {
    // the U_H x pass re-tiled by N_h columns beside the U_vW plane pass
    constexpr int TKX = L / 2 + 1;
    StridedArgs x = a.s;
    const unsigned nouter = a.nblocks / (unsigned)a.s.nchunk;
    x.nchunk = (x.ncols + TKX - 1) / TKX;
    const unsigned n1 = nouter * (unsigned)x.nchunk;
    hipLaunchKernelGGL((k_xplane_dual<L, TKX, -1, 2, 1, 1>), dim3(n1 + b.nblocks), blk_p, 0, s, x, b.z, n1);
  } else if (a.kind == FFT_PASS_STRIDED && a.sign > 0 && a.mode == 3 && db == 0 && b.mode == 2) {
    // the x pass re-tiled by N_h columns
    constexpr int TKX = L / 2 + 1;
    StridedArgs x = a.s;
    const unsigned nouter = a.nblocks / (unsigned)a.s.nchunk;
    x.nchunk = (x.ncols + TKX - 1) / TKX;
    const unsigned n1 = nouter * (unsigned)x.nchunk;
    hipLaunchKernelGGL((k_xplane_dual<L, TKX, +1, 3, 0, 2>), dim3(n1 + b.nblocks), blk_p, 0, s, x, b.z, n1);
  } else if (da == 0 && a.mode == 0 && db == 0 && b.mode == 1) {
    hipLaunchKernelGGL((k_plane_dual<L, 0, 0, 0, 1>), dim3(a.nblocks + b.nblocks), blk_p, 0, s, a.z, b.z, a.nblocks);
  } else if (da == 1 && a.mode == 0 && db == 0 && b.mode == 2) {
    hipLaunchKernelGGL((k_plane_dual<L, 1, 0, 0, 2>), dim3(a.nblocks + b.nblocks), blk_p, 0, s, a.z, b.z, a.nblocks);
  } else {
    return false;
  }
  *e = hipGetLastError();
  return true;
}

hipError_t launch_pass_any(const FftPass& ps, hipStream_t s) {
  if (ps.kind == FFT_PASS_NOP) return hipSuccess;
  if (ps.kind == FFT_PASS_ZY_R2C || ps.kind == FFT_PASS_YZ_C2R) return launch_plane(ps, s);
  switch (ps.L) {
#define X(n) \
  case n:    \
    return launch_pass<n>(ps, s);
    ARCHE_CT_SIZES(X)
#undef X
    default:
      return hipErrorNotSupported;
  }
}
int ct_z_rows(int L, int var) {
  switch (L) {
#define X(n) \
  case n:    \
    return tunable<n>() ? z_rows_var<n>(var) : z_rows<n>();
    ARCHE_CT_SIZES(X)
#undef X
    default:
      return 0;
  }
}

// chosen tile variant per (line length, pass): [0] y pass, [1] x pass, [2] z pass
int g_tile_var[3][1025];

FftPass strided_desc(int L, int mode, int sign, cplx* data, const cplx* src, const cplx* tw, int64_t es, int64_t os,
                     int nouter, int ncols, double scale, const FftFuse& f, const XGeom& g, int axis) {
  FftPass ps{};
  ps.kind = FFT_PASS_STRIDED;
  ps.L = L;
  ps.sign = sign;
  ps.mode = mode;
  ps.var = L <= 1024 ? g_tile_var[axis == 0 ? 1 : 0][L] : 0;
  const int tk = kStridedTK[ps.var];
  const int nchunk = (ncols + tk - 1) / tk;
  ps.nblocks = (unsigned)(nouter * nchunk);
  ps.s = StridedArgs{data, src, tw, es, os, ncols, nchunk, scale, f, g};
  return ps;
}
FftPass z_desc(int kind, int L, int code, const void* in, void* out, const cplx* tw, int64_t npairs, double is,
               double os, const FftFuse& f) {
  FftPass ps{};
  ps.kind = kind;
  ps.L = L;
  ps.sign = kind == FFT_PASS_Z_R2C ? -1 : +1;
  ps.mode = code;
  ps.var = L <= 1024 ? g_tile_var[2][L] : 0;
  const int B = ct_z_rows(L, ps.var);
  ps.nblocks = (unsigned)((npairs + B - 1) / B);
  ps.z = ZArgs{in, out, tw, npairs, is, os, f};
  return ps;
}

// the fused z + y pass over the Nx planes of a grid with N_y = N_z = L
FftPass plane_desc(int kind, int L, int code, const void* in, void* out, const cplx* tw, int nplanes, double is,
                   double os, const FftFuse& f) {
  FftPass ps{};
  ps.kind = kind;
  ps.L = L;
  ps.sign = kind == FFT_PASS_ZY_R2C ? -1 : +1;
  ps.mode = code;
  ps.nblocks = (unsigned)nplanes;
  ps.z = ZArgs{in, out, tw, (int64_t)nplanes * L / 2, is, os, f};
  return ps;
}
FftPass nop_desc() {
  FftPass ps{};
  ps.kind = FFT_PASS_NOP;
  return ps;
}

hipError_t ct_strided(int L, int mode, int sign, cplx* data, const cplx* src, const cplx* tw, int64_t es, int64_t os,
                      int nouter, int ncols, double scale, const FftFuse& f, const XGeom& g, int axis, hipStream_t s) {
  if (!ct_supported(L)) return hipErrorNotSupported;
  return launch_pass_any(strided_desc(L, mode, sign, data, src, tw, es, os, nouter, ncols, scale, f, g, axis), s);
}
hipError_t ct_z_r2c(int L, int fin, const double* in, cplx* out, const cplx* tw, int64_t npairs, double is, double os,
                    const FftFuse& f, hipStream_t s) {
  if (!ct_supported(L)) return hipErrorNotSupported;
  return launch_pass_any(z_desc(FFT_PASS_Z_R2C, L, fin, in, out, tw, npairs, is, os, f), s);
}
hipError_t ct_z_c2r(int L, int fout, const cplx* in, double* out, const cplx* tw, int64_t npairs, double os,
                    const FftFuse& f, hipStream_t s) {
  if (!ct_supported(L)) return hipErrorNotSupported;
  return launch_pass_any(z_desc(FFT_PASS_Z_C2R, L, fout, in, out, tw, npairs, 1.0, os, f), s);
}

Radices radices_of(const FftAxis& ax) {
  Radices r;
  r.nst = ax.nst;
  for (int i = 0; i < 8; ++i) r.r[i] = ax.radix[i];
  return r;
}

int z_rows_per_block(int Nz) {
  int B = 1536 / (Nz + 2);
  return B < 1 ? 1 : (B > 16 ? 16 : B);
}

int strided_tile(int L) { return L <= 64 ? 16 : 8; }

hipError_t strided_pass(const FftPlan* p, cplx* data, int axis, int sign, double scale, hipStream_t s) {
  const FftAxis& ax = p->ax[axis];
  const int Nx = p->N[0], Ny = p->N[1], Nh = p->Nh;
  int64_t es, os;
  int nouter;
  if (axis == 1) {  // lines along y: element stride Nh, one outer index per x
    es = Nh;
    os = (int64_t)Ny * Nh;
    nouter = Nx;
  } else {  // axis 0: lines along x, element stride Ny*Nh, the (y, k_z) plane as one run of columns
    es = (int64_t)Ny * Nh;
    os = 0;
    nouter = 1;
  }
  const int ncols = axis == 1 ? Nh : Ny * Nh;
  ProfScope prof(PROF_FFT_STRIDED, s);
  if (ct_supported(ax.L))
    return ct_strided(ax.L, 0, sign, data, data, ax.tw, es, os, nouter, ncols, scale, FftFuse{}, XGeom{}, axis, s);
  const int TK = strided_tile(ax.L);
  const int nchunk = (ncols + TK - 1) / TK;
  const size_t lds = (size_t)(2 * ax.L * TK + ax.L) * sizeof(cplx);
  hipLaunchKernelGGL(k_fft_strided, dim3(nouter * nchunk), dim3(ARCHE_BLOCK), lds, s, data, ax.tw, ax.L,
                     es, os, ncols, TK, nchunk, radices_of(ax), sign, scale);
  return hipGetLastError();
}

}  // namespace

thread_local Profiler* g_profiler = nullptr;

bool fft_size_supported(int n) {
  if (n < 2 || n > 1024 || (n & 1)) return false;
  int r = n;
  for (int p : {2, 3, 5})
    while (r % p == 0) r /= p;
  return r == 1;
}

static void factor(FftAxis& ax) {
  int r = ax.L;
  ax.nst = 0;
  while (r % 4 == 0) {
    ax.radix[ax.nst++] = 4;
    r /= 4;
  }
  while (r % 2 == 0) {
    ax.radix[ax.nst++] = 2;
    r /= 2;
  }
  while (r % 3 == 0) {
    ax.radix[ax.nst++] = 3;
    r /= 3;
  }
  while (r % 5 == 0) {
    ax.radix[ax.nst++] = 5;
    r /= 5;
  }
  for (int i = ax.nst; i < 8; ++i) ax.radix[i] = 1;
}

void fft_twiddles_host(int L, cplx* tw) {
  for (int m = 0; m < L; ++m) {
    long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
    tw[m] = cplx{(double)cosl(ang), (double)(-sinl(ang))};
  }
}

bool fft_plan_describe(FftPlan* plan, const int N[3]) {
  std::memset(plan, 0, sizeof(*plan));
  for (int a = 0; a < 3; ++a)
    if (!fft_size_supported(N[a])) return false;
  for (int a = 0; a < 3; ++a) {
    plan->N[a] = N[a];
    FftAxis& ax = plan->ax[a];
    ax.L = N[a];
    factor(ax);
    if (ax.nst > 8) return false;
  }
  plan->Nh = N[2] / 2 + 1;
  plan->ng = (int64_t)N[0] * N[1] * N[2];
  plan->nh = (int64_t)N[0] * N[1] * plan->Nh;
  return true;
}

bool fft_plan_create_with(FftPlan* plan, const int N[3], void* (*alloc)(size_t, void*),
                          void (*release)(void*, void*), void* stream) {
  if (!fft_plan_describe(plan, N)) return false;
  for (int a = 0; a < 3; ++a) {
    FftAxis& ax = plan->ax[a];
    std::vector<cplx> tw(ax.L);
    fft_twiddles_host(ax.L, tw.data());
    const size_t bytes = ax.L * sizeof(cplx);
    if (alloc) {
      ax.tw = (cplx*)alloc(bytes, stream);
      if (!ax.tw) return false;
    } else if (hipMalloc(&ax.tw, bytes) != hipSuccess) {
      return false;
    }
    if (hipMemcpy(ax.tw, tw.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
  }
  plan->ok = true;
  return true;
}

bool fft_plan_create(FftPlan* plan, const int N[3]) { return fft_plan_create_with(plan, N, nullptr, nullptr, nullptr); }

void fft_plan_destroy_with(FftPlan* plan, void (*release)(void*, void*), void* stream) {
  for (int a = 0; a < 3; ++a) {
    if (!plan->ax[a].tw) continue;
    if (release)
      release(plan->ax[a].tw, stream);
    else
      (void)hipFree(plan->ax[a].tw);
  }
  std::memset(plan, 0, sizeof(*plan));
}

void fft_plan_destroy(FftPlan* plan) { fft_plan_destroy_with(plan, nullptr, nullptr); }

// the plane passes move the real field as 16-byte pairs
static bool aligned16(const void* a, const void* b) { return (((uintptr_t)a | (uintptr_t)b) & 15u) == 0; }

hipError_t fft_r2c(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale,
                   hipStream_t s) {
  if (fft_plane_fusable(p) && aligned16(in, out)) {
    {
      ProfScope prof(PROF_FFT_Z, s);
      hipError_t e0 = launch_plane(
          plane_desc(FFT_PASS_ZY_R2C, p->N[2], 0, in, out, p->ax[2].tw, p->N[0], in_scale, 1.0, FftFuse{}), s);
      if (e0 != hipSuccess) return e0;
    }
    return strided_pass(p, out, 0, -1, out_scale, s);
  }
  const FftAxis& az = p->ax[2];
  const int Nz = p->N[2];
  const int64_t npairs = (int64_t)p->N[0] * p->N[1] / 2;
  const int B = z_rows_per_block(Nz);
  const size_t lds = (size_t)(2 * B * (Nz + 2) + Nz) * sizeof(cplx);
  {
  ProfScope prof(PROF_FFT_Z, s);
  if (ct_supported(Nz)) {
    hipError_t e0 = ct_z_r2c(Nz, 0, in, out, az.tw, npairs, in_scale, 1.0, FftFuse{}, s);
    if (e0 != hipSuccess) return e0;
  } else
  hipLaunchKernelGGL(k_fft_z_r2c, dim3((unsigned)((npairs + B - 1) / B)), dim3(ARCHE_BLOCK), lds, s, in, out,
                     az.tw, Nz, p->Nh, npairs, B, radices_of(az), in_scale, 1.0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = strided_pass(p, out, 1, -1, 1.0, s);
  if (e != hipSuccess) return e;
  return strided_pass(p, out, 0, -1, out_scale, s);
}

hipError_t fft_c2r(const FftPlan* p, cplx* in, double* out, double out_scale, hipStream_t s) {
  hipError_t e = strided_pass(p, in, 0, +1, 1.0, s);
  if (e != hipSuccess) return e;
  if (fft_plane_fusable(p) && aligned16(in, out)) {
    ProfScope prof(PROF_FFT_Z, s);
    return launch_plane(
        plane_desc(FFT_PASS_YZ_C2R, p->N[2], 0, in, out, p->ax[2].tw, p->N[0], 1.0, out_scale, FftFuse{}), s);
  }
  e = strided_pass(p, in, 1, +1, 1.0, s);
  if (e != hipSuccess) return e;
  const FftAxis& az = p->ax[2];
  const int Nz = p->N[2];
  const int64_t npairs = (int64_t)p->N[0] * p->N[1] / 2;
  const int B = z_rows_per_block(Nz);
  const size_t lds = (size_t)(2 * B * (Nz + 2) + Nz) * sizeof(cplx);
  ProfScope prof(PROF_FFT_Z, s);
  if (ct_supported(Nz)) return ct_z_c2r(Nz, 0, in, out, az.tw, npairs, out_scale, FftFuse{}, s);
  hipLaunchKernelGGL(k_fft_z_c2r, dim3((unsigned)((npairs + B - 1) / B)), dim3(ARCHE_BLOCK), lds, s, in, out,
                     az.tw, Nz, p->Nh, npairs, B, radices_of(az), out_scale);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused transforms (see fft.h).  All three line lengths need compile-time plans.
bool fft_fusable(const FftPlan* p) {
  return ct_supported(p->N[0]) && ct_supported(p->N[1]) && ct_supported(p->N[2]);
}
int fft_x_blocks(const FftPlan* p) {
  const int tk = kStridedTK[p->N[0] <= 1024 ? g_tile_var[1][p->N[0]] : 0];
  return (p->N[1] * p->Nh + tk - 1) / tk;
}
int fft_x_blocks_wide(const FftPlan* p) {
  const int tk = p->N[0] / 2 + 1;
  return (p->N[1] * p->Nh + tk - 1) / tk;
}
bool fft_x_roundtrip(int L) { return L == 128; }  // plane_len
bool fft_plane_fusable(const FftPlan* p) {
  return fft_fusable(p) && p->N[1] == p->N[2] && plane_supported(p->N[2]);
}
int fft_z_blocks(const FftPlan* p) {
  if (fft_plane_fusable(p)) return p->N[0];
  const int64_t npairs = (int64_t)p->N[0] * p->N[1] / 2;
  const int B = ct_z_rows(p->N[2], g_tile_var[2][p->N[2]]);
  return B ? (int)((npairs + B - 1) / B) : 0;
}

static XGeom xgeom(const FftPlan* p, const FftFuse& f) {
  return XGeom{p->N[0], p->N[1], p->N[2], f.L[0], f.L[1], f.L[2]};
}

bool fft_r2c_passes(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale, int fin, int fout,
                    const FftFuse& f, FftPass o[3]) {
  if (!fft_fusable(p)) return false;
  const int64_t npairs = (int64_t)p->N[0] * p->N[1] / 2;
  const int Nh = p->Nh;
  if (fft_plane_fusable(p)) {
    o[0] = plane_desc(FFT_PASS_ZY_R2C, p->N[2], fin, in, out, p->ax[2].tw, p->N[0], in_scale, 1.0, f);
    o[1] = nop_desc();
  } else {
    o[0] = z_desc(FFT_PASS_Z_R2C, p->N[2], fin, in, out, p->ax[2].tw, npairs, in_scale, 1.0, f);
    o[1] = strided_desc(p->N[1], 0, -1, out, out, p->ax[1].tw, Nh, (int64_t)p->N[1] * Nh, p->N[0], Nh, 1.0, f,
                        XGeom{}, 1);
  }
  const int mode = fout == R2C_OUT_LAP ? 1 : (fout == R2C_OUT_UH ? 2 : 0);
  o[2] = strided_desc(p->N[0], mode, -1, out, out, p->ax[0].tw, (int64_t)p->N[1] * Nh, 0, 1, p->N[1] * Nh, out_scale,
                      f, xgeom(p, f), 0);
  return true;
}

bool fft_c2r_passes(const FftPlan* p, const cplx* in, cplx* work, double* out, double out_scale, int fin, int fout,
                    const FftFuse& f, FftPass o[3]) {
  if (!fft_fusable(p)) return false;
  const int64_t npairs = (int64_t)p->N[0] * p->N[1] / 2;
  const int Nh = p->Nh;
  o[0] = strided_desc(p->N[0], fin == C2R_IN_MIX ? 3 : 0, +1, work, fin == C2R_IN_MIX ? in : work, p->ax[0].tw,
                      (int64_t)p->N[1] * Nh, 0, 1, p->N[1] * Nh, 1.0, f, xgeom(p, f), 0);
  if (fft_plane_fusable(p)) {
    o[1] = nop_desc();
    o[2] = plane_desc(FFT_PASS_YZ_C2R, p->N[2], fout, work, out, p->ax[2].tw, p->N[0], 1.0, out_scale, f);
  } else {
    o[1] = strided_desc(p->N[1], 0, +1, work, work, p->ax[1].tw, Nh, (int64_t)p->N[1] * Nh, p->N[0], Nh, 1.0, f,
                        XGeom{}, 1);
    o[2] = z_desc(FFT_PASS_Z_C2R, p->N[2], fout, work, out, p->ax[2].tw, npairs, 1.0, out_scale, f);
  }
  return true;
}

hipError_t fft_dual_launch(const FftPass& a, const FftPass& b, hipStream_t s) {
  if (a.L == b.L && a.L == 128 && plane_supported(128)) {
    ProfScope prof(plane_dir(a) >= 0 ? PROF_FFT_Z : PROF_FFT_STRIDED, s);
    hipError_t e = hipSuccess;
    if (launch_dual_L<128>(a, b, s, &e)) return e;
  }
  hipError_t e = fft_pass_launch(a, s);
  return e == hipSuccess ? fft_pass_launch(b, s) : e;
}

hipError_t fft_pass_launch(const FftPass& ps, hipStream_t s) {
  if (ps.kind == FFT_PASS_NOP) return hipSuccess;
  ProfScope prof(ps.kind == FFT_PASS_STRIDED ? PROF_FFT_STRIDED : PROF_FFT_Z, s);
  return launch_pass_any(ps, s);
}

hipError_t fft_r2c_fused(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale, int fin,
                         int fout, const FftFuse& f, hipStream_t s) {
  FftPass ps[3];
  if (!fft_r2c_passes(p, in, out, in_scale, out_scale, fin, fout, f, ps)) return hipErrorNotSupported;
  for (int i = 0; i < 3; ++i) {
    hipError_t e = fft_pass_launch(ps[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fft_c2r_fused(const FftPlan* p, const cplx* in, cplx* work, double* out, double out_scale, int fin, int fout,
                         const FftFuse& f, hipStream_t s) {
  FftPass ps[3];
  if (!fft_c2r_passes(p, in, work, out, out_scale, fin, fout, f, ps)) return hipErrorNotSupported;
  for (int i = 0; i < 3; ++i) {
    hipError_t e = fft_pass_launch(ps[i], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Tile autotuner (fft.h).
static std::mutex g_tune_mtx;
static bool g_tuned[3][1025];

int fft_tile_variant(int pass, int L, int force) {
  if (pass < 0 || pass > 2 || L < 0 || L > 1024) return -1;
  std::lock_guard<std::mutex> lk(g_tune_mtx);
  if (force >= 0 && force <= 2 && (force == 0 || (ct_supported(L) && L > 96))) {
    g_tile_var[pass][L] = force;
    g_tuned[pass][L] = true;
  }
  return g_tile_var[pass][L];
}

hipError_t fft_tune(const FftPlan* p, cplx* scratch_c, double* scratch_r, hipStream_t s) {
  const char* env = getenv("ARCHE_FFT_TUNE");
  if (env && env[0] == '0') return hipSuccess;
  std::lock_guard<std::mutex> lk(g_tune_mtx);
  const int Nh = p->Nh;
  const int64_t npairs = (int64_t)p->N[0] * p->N[1] / 2;
  const int Ls[3] = {p->N[1], p->N[0], p->N[2]};
  bool any = false;
  for (int pass = 0; pass < 3; ++pass)
    any = any || (Ls[pass] > 96 && ct_supported(Ls[pass]) && !g_tuned[pass][Ls[pass]]);
  if (!any) return hipSuccess;
  hipError_t e = hipMemsetAsync(scratch_c, 0, p->nh * sizeof(cplx), s);
  if (e == hipSuccess) e = hipMemsetAsync(scratch_r, 0, p->ng * sizeof(double), s);
  hipEvent_t t0, t1;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(t0);
    return e;
  }
  for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
    const int L = Ls[pass];
    if (L <= 96 || !ct_supported(L) || g_tuned[pass][L]) continue;
    if (pass == 1 && fft_plane_fusable(p)) {
      // on plane-pass grids the SCF iteration's x passes run re-tiled beside
      // plane passes or, the Laplacian round trips, alone, where the variants
      // time within noise of each other: keep the default tile
      g_tile_var[pass][L] = 0;
      g_tuned[pass][L] = true;
      continue;
    }
    float best_ms = 0.f;
    int best = 0;
    for (int v = 0; v < 3 && e == hipSuccess; ++v) {
      g_tile_var[pass][L] = v;
      FftPass ps;
      if (pass == 0)
        ps = strided_desc(L, 0, -1, scratch_c, scratch_c, p->ax[1].tw, Nh, (int64_t)p->N[1] * Nh, p->N[0], Nh, 1.0,
                          FftFuse{}, XGeom{}, 1);
      else if (pass == 1)
        ps = strided_desc(L, 0, -1, scratch_c, scratch_c, p->ax[0].tw, (int64_t)p->N[1] * Nh, 0, 1, p->N[1] * Nh,
                          1.0, FftFuse{}, XGeom{}, 0);
      else
        ps = z_desc(FFT_PASS_Z_R2C, L, 0, scratch_r, scratch_c, p->ax[2].tw, npairs, 1.0, 1.0, FftFuse{});
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_pass_any(ps, s);
      // the best of three timings of 20 launches: one pass takes some 10 us, so
      // single short timings are at the mercy of event jitter
      float ms = 0.f;
      for (int trial = 0; trial < 3 && e == hipSuccess; ++trial) {
        e = hipEventRecord(t0, s);
        for (int w = 0; w < 20 && e == hipSuccess; ++w) e = launch_pass_any(ps, s);
        if (e == hipSuccess) e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, t0, t1);
        if (e == hipSuccess && (trial == 0 || t < ms)) ms = t;
      }
      if (e != hipSuccess) break;
      // a variant must beat the default by 5% to be taken
      if (v == 0 || ms < 0.95f * best_ms) {
        if (v == 0 || ms < best_ms) {
          best_ms = ms;
          best = v;
        }
      }
    }
    g_tile_var[pass][L] = e == hipSuccess ? best : 0;
    g_tuned[pass][L] = true;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  return e;
}
