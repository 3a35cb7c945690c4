// Tile bodies of the compile-time FFT passes (fft_plans.h), shared by the
// single-grid kernels (fft.hip) and the batched ones (fft_batch.hip): both run
// the same code per tile, so a batched transform is bit-identical to a single one.
#pragma once

#include "fft.h"
#include "fft_plans.h"

namespace fftct {

struct ColIn {  // column tile of a strided pass: element k of column `line`
  const cplx* base;
  int64_t es;
  int nc;
  __device__ cplx operator()(int line, int k) const { return line < nc ? base[(int64_t)k * es + line] : cplx{0.0, 0.0}; }
};
struct ColOut {
  cplx* base;
  int64_t es;
  int nc;
  double scale;
  __device__ void operator()(int line, int k, cplx v) const {
    if (line < nc) base[(int64_t)k * es + line] = cscale(v, scale);
  }
  __device__ void barrier_before() const {}
  __device__ void barrier_after() const {}
};

struct ColOutLap {  // R2C_OUT_LAP
  cplx* base;
  int64_t es;
  int nc;
  double scale;
  XGeom g;
  int o, c0;
  __device__ void operator()(int line, int k, cplx v) const {
    if (line >= nc) return;
    const double q2 = 39.478417604357434 * g.k2c(k, c0 + line);  // (2 pi)^2 |k|^2
    base[(int64_t)k * es + line] = cscale(v, -q2 * scale);
  }
  __device__ void barrier_before() const {}
  __device__ void barrier_after() const {}
};

struct ColOutUH {  // R2C_OUT_UH
  cplx* base;
  const cplx* nhat_i;
  int64_t es;
  int nc;
  double scale;
  XGeom g;
  int o, c0;
  double* acc;
  __device__ void operator()(int line, int k, cplx v) const {
    if (line >= nc) return;
    const int64_t at = (int64_t)k * es + line;
    const cplx a = cscale(v, scale);
    base[at] = a;
    const double k2 = g.k2c(k, c0 + line);
    if (k2 > 0.0) {
      const cplx d = csub(nhat_i[at], a);
      *acc += g.weightc(c0 + line) * (d.x * d.x + d.y * d.y) / (3.14159265358979323846 * k2);
    }
  }
  __device__ void barrier_before() const {}
  __device__ void barrier_after() const {}
};

struct ColInMix {  // C2R_IN_MIX: n_o^ = a + w (nhat_i - a); nhat_i <- n_o^; value n_o^/(pi k^2)
  const cplx* a;
  cplx* nhat_i;
  int64_t es;
  int nc;
  double w;
  XGeom g;
  int o, c0;
  __device__ cplx operator()(int line, int k) const {
    if (line >= nc) return cplx{0.0, 0.0};
    const int64_t at = (int64_t)k * es + line;
    const cplx x = a[at];
    const cplx no = cadd(x, cscale(csub(nhat_i[at], x), w));
    nhat_i[at] = no;
    const double k2 = g.k2c(k, c0 + line);
    return k2 > 0.0 ? cscale(no, 1.0 / (3.14159265358979323846 * k2)) : cplx{0.0, 0.0};
  }
};

struct LdsLap {  // MODE 4: the forward result times -(2 pi |k|)^2 scale, back into LDS
  cplx* buf;
  double scale;
  XGeom g;
  int o, c0, TK;
  __device__ void operator()(int line, int k, cplx v) const {
    const double q2 = 39.478417604357434 * g.k2c(k, c0 + line);  // (2 pi)^2 |k|^2
    buf[k * TK + line] = cscale(v, -q2 * scale);
  }
  __device__ void barrier_before() const { __syncthreads(); }
  __device__ void barrier_after() const { __syncthreads(); }
};

// One tile (block `bid` of the pass).  MODE 0: plain pass.  MODE 1/2/3: x pass
// with R2C_OUT_LAP / R2C_OUT_UH / C2R_IN_MIX.  MODE 4: the x pass of R2C with
// the Laplacian followed by the x pass of the C2R that comes back from it, in
// one pass: forward along the line, times -(2 pi |k|)^2 scale, inverse, store.
template <int L, int TK, int S, int MODE, int NT = ARCHE_BLOCK>
__device__ inline void strided_body(const StridedArgs& A, unsigned bid, cplx* lds, cplx* tw, double* sh) {
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = A.tw[i];
  __syncthreads();
  const int o = (int)bid / A.nchunk;
  const int c0 = ((int)bid - o * A.nchunk) * TK;
  const int nc = (A.ncols - c0) < TK ? (A.ncols - c0) : TK;
  cplx* base = A.data + (int64_t)o * A.os + c0;
  const int64_t es = A.es;
  if constexpr (MODE == 0) {
    run<L, TK, NT, true, S, 1>(ColIn{base, es, nc}, ColOut{base, es, nc, A.scale}, lds, tw, nc,
                                         typename Plan<L>::R{});
  } else if constexpr (MODE == 1) {
    run<L, TK, NT, true, S, 1>(ColIn{base, es, nc}, ColOutLap{base, es, nc, A.scale, A.g, o, c0}, lds, tw,
                                         nc, typename Plan<L>::R{});
  } else if constexpr (MODE == 2) {
    double acc = 0.0;
    run<L, TK, NT, true, S, 1>(
        ColIn{base, es, nc}, ColOutUH{base, A.f.nhat_i + (int64_t)o * A.os + c0, es, nc, A.scale, A.g, o, c0, &acc},
        lds, tw, nc, typename Plan<L>::R{});
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) A.f.partials[bid] = acc;
  } else if constexpr (MODE == 3) {
    const int64_t off = (int64_t)o * A.os + c0;
    run<L, TK, NT, true, S, 1>(ColInMix{A.src + off, A.f.nhat_i + off, es, nc, *A.f.w, A.g, o, c0},
                                         ColOut{base, es, nc, A.scale}, lds, tw, nc, typename Plan<L>::R{});
  } else {
    static_assert(MODE == 4, "modes 0-4");
    static_assert(nstages(typename Plan<L>::R{}) > 1, "the tile is staged in LDS");
    run<L, TK, NT, true, -1, 1>(ColIn{base, es, nc}, LdsLap{lds, A.scale, A.g, o, c0, TK}, lds, tw, nc,
                                typename Plan<L>::R{});
    run<L, TK, NT, true, +1, 1>(LdsIO<L, TK, true>{lds}, ColOut{base, es, nc, 1.0}, lds, tw, nc,
                                typename Plan<L>::R{});
  }
}
template <int L, int TK>
constexpr int strided_lds() {
  return nstages(typename Plan<L>::R{}) > 1 ? lds_size<L, TK, true>() : 1;
}

struct PairIn {  // two real rows packed as one complex line
  const double* src;
  int L;
  int nv;
  double s;
  __device__ cplx operator()(int line, int k) const {
    if (line >= nv) return cplx{0.0, 0.0};
    const double* r0 = src + (int64_t)line * 2 * L;
    return cplx{r0[k] * s, r0[L + k] * s};
  }
};
struct PairInSqrt {  // R2C_IN_SQRT
  const double* src;
  int L;
  int nv;
  double s;
  __device__ cplx operator()(int line, int k) const {
    if (line >= nv) return cplx{0.0, 0.0};
    const double* r0 = src + (int64_t)line * 2 * L;
    return cplx{sqrt(r0[k]) * s, sqrt(r0[L + k]) * s};
  }
};
struct PairInMix {  // R2C_IN_MIX_SQRT: n_o = n_a + w (n_i - n_a); n_i <- n_o; sqrt(n_o)
  const double* na;
  double* ni;
  int L;
  int nv;
  double s, w;
  __device__ double one(int64_t at) const {
    const double a = na[at];
    const double o = a + w * (ni[at] - a);
    ni[at] = o;
    return sqrt(o) * s;
  }
  __device__ cplx operator()(int line, int k) const {
    if (line >= nv) return cplx{0.0, 0.0};
    const int64_t at = (int64_t)line * 2 * L + k;
    return cplx{one(at), one(at + L)};
  }
};

template <int L, int B, int FIN, int NT = ARCHE_BLOCK>
__device__ inline void z_r2c_body(const ZArgs& A, unsigned bid, cplx* lds, cplx* tw) {
  constexpr int Nh = L / 2 + 1;
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = A.tw[i];
  __syncthreads();
  const double* in = (const double*)A.in;
  const int64_t p0 = (int64_t)bid * B;
  const int nb = (int)((A.npairs - p0) < B ? (A.npairs - p0) : B);
  LdsIO<L, B, false> res{lds};
  if constexpr (FIN == 0)
    run<L, B, NT, false, -1, 1>(PairIn{in + p0 * 2 * L, L, nb, A.in_scale}, res, lds, tw, nb,
                                          typename Plan<L>::R{});
  else if constexpr (FIN == 1)
    run<L, B, NT, false, -1, 1>(PairInSqrt{in + p0 * 2 * L, L, nb, A.in_scale}, res, lds, tw, nb,
                                          typename Plan<L>::R{});
  else
    run<L, B, NT, false, -1, 1>(PairInMix{in + p0 * 2 * L, A.f.n_i + p0 * 2 * L, L, nb, A.in_scale, *A.f.w},
                                          res, lds, tw, nb, typename Plan<L>::R{});
  cplx* dst = (cplx*)A.out + p0 * 2 * Nh;
  for (int q = threadIdx.x; q < nb * 2 * Nh; q += NT) {
    const int l = q / (2 * Nh);
    const int w = q - l * 2 * Nh;
    const int r = w / Nh;
    const int k = w - r * Nh;
    const cplx zk = res(l, k);
    const cplx zn = res(l, k == 0 ? 0 : L - k);
    cplx v;
    if (r == 0)
      v = cplx{0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y)};
    else
      v = cplx{0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x)};
    dst[q] = cscale(v, A.out_scale);
  }
}
template <int L, int B>
constexpr int z_r2c_lds() {
  return lds_size<L, B, false>();
}

struct HermIn {  // Z_k = X_k + i Y_k from the half spectra of two real rows
  const cplx* src;
  int L, Nh, nv;
  __device__ cplx operator()(int line, int k) const {
    if (line >= nv) return cplx{0.0, 0.0};
    const cplx* X = src + (int64_t)line * 2 * Nh;
    const cplx* Y = X + Nh;
    cplx x, y;
    if (k == 0 || 2 * k == L) {
      x = cplx{X[k].x, 0.0};
      y = cplx{Y[k].x, 0.0};
    } else if (2 * k < L) {
      x = X[k];
      y = Y[k];
    } else {
      x = cconj(X[L - k]);
      y = cconj(Y[L - k]);
    }
    return cplx{x.x - y.y, x.y + y.x};
  }
};
struct PairOut {
  double* dst;
  int L, nv;
  double scale;
  __device__ void operator()(int line, int k, cplx v) const {
    if (line >= nv) return;
    double* r0 = dst + (int64_t)line * 2 * L;
    r0[k] = v.x * scale;
    r0[L + k] = v.y * scale;
  }
  __device__ void barrier_before() const {}
  __device__ void barrier_after() const {}
};

struct PairOutUvw {  // C2R_OUT_UVW: accumulate (v_vW[n_i] - v_vW[n_a]) (n_i - n_a), no store
  const double* ni;
  const double* lapi;
  const double* na;
  const double* w;  // (n_i - n_a)/sqrt(n_a) with the v_vW[n_i] part summed elsewhere, or null
  int L, nv;
  double scale, hl;  // hl = lambda/2
  double* acc;
  __device__ void one(int64_t at, double lap) const {
    if (w) {
      *acc += hl * lap * w[at];
      return;
    }
    const double a = ni[at], b = na[at];
    const double vi = -hl * lapi[at] / sqrt(a);
    const double va = -hl * lap / sqrt(b);
    *acc += (vi - va) * (a - b);
  }
  __device__ void operator()(int line, int k, cplx v) const {
    if (line >= nv) return;
    const int64_t at = (int64_t)line * 2 * L + k;
    one(at, v.x * scale);
    one(at + L, v.y * scale);
  }
  __device__ void barrier_before() const {}
  __device__ void barrier_after() const {}
};

template <int L, int B, int FOUT, int NT = ARCHE_BLOCK>
__device__ inline void z_c2r_body(const ZArgs& A, unsigned bid, cplx* lds, cplx* tw, double* sh) {
  constexpr int Nh = L / 2 + 1;
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = A.tw[i];
  __syncthreads();
  const cplx* in = (const cplx*)A.in;
  const int64_t p0 = (int64_t)bid * B;
  const int nb = (int)((A.npairs - p0) < B ? (A.npairs - p0) : B);
  if constexpr (FOUT == 0) {
    run<L, B, NT, false, +1, 1>(HermIn{in + p0 * 2 * Nh, L, Nh, nb},
                                          PairOut{(double*)A.out + p0 * 2 * L, L, nb, A.out_scale}, lds, tw, nb,
                                          typename Plan<L>::R{});
  } else {
    double acc = 0.0;
    const int64_t off = p0 * 2 * L;
    run<L, B, NT, false, +1, 1>(
        HermIn{in + p0 * 2 * Nh, L, Nh, nb},
        PairOutUvw{A.f.n_i + off, A.f.lap_i + off, A.f.n_a + off, A.f.uvw_w ? A.f.uvw_w + off : nullptr, L, nb,
                   A.out_scale, 0.5 * A.f.lam, &acc}, lds, tw,
        nb, typename Plan<L>::R{});
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) A.f.partials[bid] = acc;
  }
}
template <int L, int B>
constexpr int z_c2r_lds() {
  return nstages(typename Plan<L>::R{}) > 1 ? lds_size<L, B, false>() : 1;
}

constexpr int CT_TK = 16;
template <int L>
constexpr int ct_rows() {
  return L >= 96 ? 16 : 32;
}

}  // namespace fftct

namespace fftct {

// ---------------------------------------------------------------------------
// Plane passes for grids with N_y = N_z = L: one block per x plane holds the
// whole plane (L x (L/2+1) complex) in LDS, so the z and y transforms of a 3D
// transform run in one pass that reads and writes the plane once.

template <int L>
constexpr int plane_elems() {
  return L * (L / 2 + 1);
}
// LDS of a plane pass: the plane, or its L/2 row pairs in the padded row layout
template <int L>
constexpr int plane_lds() {
  return plane_elems<L>() > (L / 2) * row_pitch<L>() ? plane_elems<L>() : (L / 2) * row_pitch<L>();
}

struct PlaneOut {  // element (k_y = k, k_z = line) of the plane in global memory
  cplx* base;
  int nh;
  double scale;
  __device__ void operator()(int line, int k, cplx v) const { base[(int64_t)k * nh + line] = cscale(v, scale); }
  __device__ void barrier_before() const {}
  __device__ void barrier_after() const {}
};

// The real plane in LDS: row pair l (rows y = 2l, 2l+1) at doubles
// [l*RP, l*RP + 2L), RP = 2L + 4 (the pad staggers the LDS banks of
// neighbouring pairs); it fills exactly the space of the complex plane.
template <int L>
constexpr int real_pair_pitch() {
  return 2 * L + 4;
}
template <int L>
struct RealPairsIn {  // two real rows packed as one complex line, from LDS
  const double* r;
  __device__ cplx operator()(int line, int k) const {
    const double* r0 = r + line * real_pair_pitch<L>();
    return cplx{r0[k], r0[L + k]};
  }
};
template <int L>
struct RealPairsOut {  // the inverse: line -> rows 2l, 2l+1 in LDS (in place, so a barrier first)
  double* r;
  double scale;
  __device__ void operator()(int line, int k, cplx v) const {
    double* r0 = r + line * real_pair_pitch<L>();
    r0[k] = v.x * scale;
    r0[L + k] = v.y * scale;
  }
  __device__ void barrier_before() const { __syncthreads(); }
  __device__ void barrier_after() const { __syncthreads(); }
};
// LDS double index of plane element q = y*L + z (the global row-major order)
template <int L>
__device__ inline int real_at(int q) {
  const int y = q / L, z = q - (q / L) * L;
  return (y >> 1) * real_pair_pitch<L>() + (y & 1) * L + z;
}

// Element (k_z = line, y = k) of the half plane from the z transforms of the row
// pairs (Z = X + i Y for rows 2l, 2l+1): X_k = (Z_k + conj Z_{L-k})/2,
// Y_k = (Z_k - conj Z_{L-k})/(2i).
template <int L>
struct SplitIn {
  LdsIO<L, L / 2, false> packed;
  __device__ cplx operator()(int line, int k) const {
    const cplx zk = packed(k >> 1, line);
    const cplx zn = packed(k >> 1, line == 0 ? 0 : L - line);
    return (k & 1) ? cplx{0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x)} : cplx{0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y)};
  }
};

// R2C: the real plane is read once with coalesced 16-byte loads (input transform
// FIN as in the z pass applied on the way) into LDS; z transform of its L/2 row
// pairs; y transform of the Hermitian split (formed as the first stage loads),
// store.
template <int L, int FIN, int NT>
__device__ inline void zy_r2c_body(const ZArgs& A, unsigned bid, cplx* plane, cplx* tw) {
  constexpr int Nh = L / 2 + 1;
  constexpr int NP = L / 2;
  static_assert(lds_size<L, NP, false>() <= plane_lds<L>(), "packed rows fit the plane's LDS");
  static_assert(NP * real_pair_pitch<L>() <= 2 * plane_lds<L>(), "real rows fit the plane's LDS");
  static_assert(L % 2 == 0, "pairs of doubles");
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = A.tw[i];
  const int64_t off = (int64_t)bid * L * L;
  const double2* in2 = (const double2*)((const double*)A.in + off);
  double* rl = (double*)plane;
  constexpr int N2 = L * L / 2;
  for (int q = threadIdx.x; q < N2; q += NT) {
    double2 v = in2[q];
    if constexpr (FIN == 1) {
      v.x = sqrt(v.x);
      v.y = sqrt(v.y);
    } else if constexpr (FIN == 2) {
      double2* ni2 = (double2*)(A.f.n_i + off);
      const double2 b = ni2[q];
      const double w = *A.f.w;
      v.x = v.x + w * (b.x - v.x);
      v.y = v.y + w * (b.y - v.y);
      ni2[q] = v;
      v.x = sqrt(v.x);
      v.y = sqrt(v.y);
    }
    const int at = real_at<L>(2 * q);  // 2q and 2q+1 share a row (L even)
    rl[at] = v.x * A.in_scale;
    rl[at + 1] = v.y * A.in_scale;
  }
  __syncthreads();
  LdsIO<L, NP, false> packed{plane};
  run<L, NP, NT, false, -1, 1>(RealPairsIn<L>{rl}, packed, plane, tw, NP, typename Plan<L>::R{});
  // the y transform reads the rows 2l, 2l+1 split out of pair l as it loads
  // (its first stage has read everything before it overwrites the pairs)
  constexpr int NOUT = L * Nh;
  run<L, Nh, NT, true, -1, 1>(SplitIn<L>{packed}, PlaneOut{(cplx*)A.out + (int64_t)bid * NOUT, Nh, A.out_scale},
                              plane, tw, Nh, typename Plan<L>::R{});
}

// C2R: y transform of the plane into LDS, then the z transform of its row pairs,
// whose last stage stores the real plane (FOUT = 0); for FOUT = 1 the real plane
// goes to LDS and one coalesced pass forms the U_vW partial sum instead.
template <int L, int FOUT, int NT>
__device__ inline void yz_c2r_body(const ZArgs& A, unsigned bid, cplx* plane, cplx* tw, double* sh) {
  constexpr int Nh = L / 2 + 1;
  constexpr int NP = L / 2;
  for (int i = threadIdx.x; i < L; i += NT) tw[i] = A.tw[i];
  __syncthreads();
  const cplx* in = (const cplx*)A.in + (int64_t)bid * L * Nh;
  LdsIO<L, Nh, true> pl{plane};
  run<L, Nh, NT, true, +1, 1>(ColIn{in, Nh, Nh}, pl, plane, tw, Nh, typename Plan<L>::R{});
  const int64_t off = (int64_t)bid * L * L;
  if constexpr (FOUT == 0) {
    // the z transform's last stage stores the row pairs straight to the plane
    run<L, NP, NT, false, +1, 1>(HermIn{plane, L, Nh, NP}, PairOut{(double*)A.out + off, L, NP, A.out_scale}, plane,
                                 tw, NP, typename Plan<L>::R{});
  } else {
    double* rl = (double*)plane;
    run<L, NP, NT, false, +1, 1>(HermIn{plane, L, Nh, NP}, RealPairsOut<L>{rl, A.out_scale}, plane, tw, NP,
                                 typename Plan<L>::R{});
    constexpr int N2 = L * L / 2;
    // (v_vW[n_i] - v_vW[n_a]) (n_i - n_a) with v_vW[n] = -(lambda/2) lap / sqrt(n);
    // with uvw_w the SCF kernel has summed the v_vW[n_i] part and left
    // (n_i - n_a)/sqrt(n_a), so this pass reads one field
    const double hl = 0.5 * A.f.lam;
    double acc = 0.0;
    if (A.f.uvw_w) {
      const double2* w2 = (const double2*)(A.f.uvw_w + off);
      for (int q = threadIdx.x; q < N2; q += NT) {
        const int at = real_at<L>(2 * q);
        const double2 w = w2[q];
        acc += hl * rl[at] * w.x;
        acc += hl * rl[at + 1] * w.y;
      }
    } else {
      const double2* ni2 = (const double2*)(A.f.n_i + off);
      const double2* li2 = (const double2*)(A.f.lap_i + off);
      const double2* na2 = (const double2*)(A.f.n_a + off);
      for (int q = threadIdx.x; q < N2; q += NT) {
        const int at = real_at<L>(2 * q);
        const double2 a = ni2[q], li = li2[q], b = na2[q];
        acc += (-hl * li.x / sqrt(a.x) + hl * rl[at] / sqrt(b.x)) * (a.x - b.x);
        acc += (-hl * li.y / sqrt(a.y) + hl * rl[at + 1] / sqrt(b.y)) * (a.y - b.y);
      }
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) A.f.partials[bid] = acc;
  }
}

}  // namespace fftct
