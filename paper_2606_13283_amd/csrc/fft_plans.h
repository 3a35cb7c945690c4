// Compile-time FFT kernels for the line lengths the grids use.  Each size has a
// fixed radix plan; every butterfly is unrolled in registers, the first stage
// reads its inputs straight from global memory and the last stage writes its
// outputs straight back, and the stages in between exchange through a single
// LDS buffer (registers carry the values across the barrier).  All index
// arithmetic folds to constants.
#pragma once

#include "common.h"

namespace fftct {

__device__ inline cplx mul_si(cplx z, double s) { return cplx{-s * z.y, s * z.x}; }  // (s i) z

template <int S>
__device__ inline void b2(cplx* v) {
  cplx a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <int S>
__device__ inline void b3(cplx* v) {
  const double H = 0.86602540378443864676;  // sqrt(3)/2
  cplx a = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
  cplx m = cplx{a.x - 0.5 * s.x, a.y - 0.5 * s.y};
  cplx t = mul_si(cscale(d, H), (double)S);
  v[0] = cadd(a, s);
  v[1] = cadd(m, t);
  v[2] = csub(m, t);
}
template <int S>
__device__ inline void b4(cplx* v) {
  cplx t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  cplx t2 = cadd(v[1], v[3]), t3 = mul_si(csub(v[1], v[3]), (double)S);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}
template <int S>
__device__ inline void b5(cplx* v) {
  const double C1 = 0.30901699437494742410, C2 = -0.80901699437494742410;
  const double S1 = 0.95105651629515357212, S2 = 0.58778525229247312917;
  cplx a = v[0];
  cplx s1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
  cplx s2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
  cplx r1 = cplx{a.x + C1 * s1.x + C2 * s2.x, a.y + C1 * s1.y + C2 * s2.y};
  cplx r2 = cplx{a.x + C2 * s1.x + C1 * s2.x, a.y + C2 * s1.y + C1 * s2.y};
  cplx i1 = mul_si(cplx{S1 * d1.x + S2 * d2.x, S1 * d1.y + S2 * d2.y}, (double)S);
  cplx i2 = mul_si(cplx{S2 * d1.x - S1 * d2.x, S2 * d1.y - S1 * d2.y}, (double)S);
  v[0] = cadd(a, cadd(s1, s2));
  v[1] = cadd(r1, i1);
  v[4] = csub(r1, i1);
  v[2] = cadd(r2, i2);
  v[3] = csub(r2, i2);
}
// radix 8 = 2 x 4: X_{2m} = DFT4(x_n + x_{n+4}), X_{2m+1} = DFT4((x_n - x_{n+4}) W8^n)
template <int S>
__device__ inline void b8(cplx* v) {
  const double C = 0.70710678118654752440;
  cplx a[4], b[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    a[n] = cadd(v[n], v[n + 4]);
    b[n] = csub(v[n], v[n + 4]);
  }
  b[1] = cmul(b[1], cplx{C, S * C});
  b[2] = mul_si(b[2], (double)S);
  b[3] = cmul(b[3], cplx{-C, S * C});
  b4<S>(a);
  b4<S>(b);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    v[2 * m] = a[m];
    v[2 * m + 1] = b[m];
  }
}
// radix 16 = 2 x 8 with twiddles W16^n
template <int S>
__device__ inline void b16(cplx* v) {
  const double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, c2 = 0.70710678118654752440;
  const double cs[8] = {1.0, c1, c2, s1, 0.0, -s1, -c2, -c1};
  const double sn[8] = {0.0, s1, c2, c1, 1.0, c1, c2, s1};
  cplx a[8], b[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    a[n] = cadd(v[n], v[n + 8]);
    b[n] = csub(v[n], v[n + 8]);
    if (n) b[n] = cmul(b[n], cplx{cs[n], S * sn[n]});
  }
  b8<S>(a);
  b8<S>(b);
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    v[2 * m] = a[m];
    v[2 * m + 1] = b[m];
  }
}
template <int R, int S>
__device__ inline void bfly(cplx* v) {
  if constexpr (R == 2) b2<S>(v);
  else if constexpr (R == 3) b3<S>(v);
  else if constexpr (R == 4) b4<S>(v);
  else if constexpr (R == 5) b5<S>(v);
  else if constexpr (R == 8) b8<S>(v);
  else b16<S>(v);
}

template <int... Rs>
struct RList {};

template <int L>
struct Plan;  // radices whose product is L
#define ARCHE_FFT_PLAN(L, ...) \
  template <>                  \
  struct Plan<L> {             \
    using R = RList<__VA_ARGS__>; \
  };
ARCHE_FFT_PLAN(16, 16)
ARCHE_FFT_PLAN(20, 4, 5)
ARCHE_FFT_PLAN(24, 8, 3)
ARCHE_FFT_PLAN(30, 2, 3, 5)
ARCHE_FFT_PLAN(32, 8, 4)
ARCHE_FFT_PLAN(40, 8, 5)
ARCHE_FFT_PLAN(48, 16, 3)
ARCHE_FFT_PLAN(50, 2, 5, 5)
ARCHE_FFT_PLAN(54, 2, 3, 3, 3)
ARCHE_FFT_PLAN(60, 4, 3, 5)
ARCHE_FFT_PLAN(64, 8, 8)
ARCHE_FFT_PLAN(72, 8, 3, 3)
ARCHE_FFT_PLAN(80, 16, 5)
ARCHE_FFT_PLAN(96, 8, 4, 3)
ARCHE_FFT_PLAN(100, 4, 5, 5)
ARCHE_FFT_PLAN(120, 8, 3, 5)
ARCHE_FFT_PLAN(128, 16, 8)
ARCHE_FFT_PLAN(144, 16, 3, 3)
ARCHE_FFT_PLAN(160, 16, 2, 5)
ARCHE_FFT_PLAN(180, 4, 3, 3, 5)
ARCHE_FFT_PLAN(192, 16, 4, 3)
ARCHE_FFT_PLAN(256, 16, 16)
#undef ARCHE_FFT_PLAN

// ---------------------------------------------------------------------------
// Lines of a tile are addressed through small accessor objects:
//   ld(line, k)  -> input element k of `line` (first stage)
//   st(line, k, v)  output element k of `line` (last stage)
// Each thread handles butterflies t = threadIdx.x + NT*p; LINE_FAST maps
// consecutive threads to consecutive lines (for column tiles), otherwise to
// consecutive butterflies of one line (for contiguous rows).

template <int L, int NL, int NT, bool LINE_FAST, int R>
struct StageGeom {
  static constexpr int nb = L / R;
  static constexpr int total = nb * NL;
  static constexpr int PER = (total + NT - 1) / NT;
  __device__ static inline void idx(int t, int& line, int& j) {
    if (LINE_FAST) {
      line = t % NL;
      j = t / NL;
    } else {
      j = t % nb;
      line = t / nb;
    }
  }
};

// LDS element k of line `line`: line-interleaved layout for column tiles,
// line-contiguous for row tiles.  A row tile's first stage writes each
// butterfly's R0 outputs (R0 the plan's first radix) to consecutive elements,
// so the lanes of one line store R0 elements apart, on the same LDS banks when
// R0 >= 4: one complex of padding after every R0 elements spreads them over the
// banks (and one more per line staggers neighbouring lines).
template <int R, int... Rs>
constexpr int first_radix(RList<R, Rs...>) {
  return R;
}
template <int L>
constexpr int row_pad() {
  return first_radix(typename Plan<L>::R{}) >= 4 ? first_radix(typename Plan<L>::R{}) : 0;
}
template <int L>
constexpr int row_pitch() {
  return L + (row_pad<L>() ? L / row_pad<L>() : 0) + 1;
}
template <int L, int NL, bool LINE_FAST>
__device__ inline int lds_at(int line, int k) {
  if constexpr (LINE_FAST) return k * NL + line;
  else return line * row_pitch<L>() + k + (row_pad<L>() ? k / row_pad<L>() : 0);
}
template <int L, int NL, bool LINE_FAST>
constexpr int lds_size() {
  return LINE_FAST ? L * NL : NL * row_pitch<L>();
}

// One Stockham stage: inputs from `In`, outputs to `Out`; twiddles from LDS table
// tw[m] = exp(-2 pi i m / L) (conjugated for the inverse).
template <int L, int NL, int NT, bool LINE_FAST, int R, int Ns, int S, class In, class Out>
__device__ inline void stage(const In& in, const Out& out, const cplx* tw, int nlines_valid) {
  using G = StageGeom<L, NL, NT, LINE_FAST, R>;
  constexpr int tstep = L / (Ns * R);
  cplx v[G::PER][R];
#pragma unroll
  for (int p = 0; p < G::PER; ++p) {
    const int t = threadIdx.x + NT * p;
    if (G::total % NT == 0 || t < G::total) {
      int line, j;
      G::idx(t, line, j);
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = in(line, j + r * G::nb);
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx w = tw[r * k * tstep];
          if (S > 0) w.y = -w.y;
          v[p][r] = cmul(v[p][r], w);
        }
      }
      bfly<R, S>(v[p]);
    }
  }
  out.barrier_before();
#pragma unroll
  for (int p = 0; p < G::PER; ++p) {
    const int t = threadIdx.x + NT * p;
    if (G::total % NT == 0 || t < G::total) {
      int line, j;
      G::idx(t, line, j);
      const int k = j % Ns;
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) out(line, base + r * Ns, v[p][r]);
    }
  }
  out.barrier_after();
}

template <int L, int NL, bool LINE_FAST>
struct LdsIO {
  cplx* buf;
  __device__ cplx operator()(int line, int k) const { return buf[lds_at<L, NL, LINE_FAST>(line, k)]; }
  __device__ void operator()(int line, int k, cplx v) const { buf[lds_at<L, NL, LINE_FAST>(line, k)] = v; }
  __device__ void barrier_before() const { __syncthreads(); }  // all reads of this stage are done
  __device__ void barrier_after() const { __syncthreads(); }   // all writes are visible
};

// Run stages R0, Rs... (Ns = product so far).  The first reads `in`, the last
// writes `out`, the rest go through LDS.
template <int L, int NL, int NT, bool LINE_FAST, int S, int Ns, class In, class Out, int R>
__device__ inline void run(const In& in, const Out& out, cplx* lds, const cplx* tw, int nv, RList<R>) {
  stage<L, NL, NT, LINE_FAST, R, Ns, S>(in, out, tw, nv);
}
template <int L, int NL, int NT, bool LINE_FAST, int S, int Ns, class In, class Out, int R, int R2, int... Rest>
__device__ inline void run(const In& in, const Out& out, cplx* lds, const cplx* tw, int nv, RList<R, R2, Rest...>) {
  LdsIO<L, NL, LINE_FAST> mid{lds};
  stage<L, NL, NT, LINE_FAST, R, Ns, S>(in, mid, tw, nv);
  run<L, NL, NT, LINE_FAST, S, Ns * R>(mid, out, lds, tw, nv, RList<R2, Rest...>{});
}

template <int... Rs>
constexpr int nstages(RList<Rs...>) {
  return sizeof...(Rs);
}

}  // namespace fftct
