// Learned initial density: a 3D U-Net (constant width 32, four levels, periodic
// 3x3x3 convolutions, 2x2x2 mean pooling, nearest upsampling with additive
// skips, 1x1x1 input/output layers) that corrects the one-center guess of the
// SCF (Sec. 2.5.1) from [one-center guess, previous converged density].
//
// Tensors are channels-last BF16, [D][H][W][32] (one point = 64 contiguous
// bytes).  The 3x3x3 convolutions run on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulate) as implicit GEMMs:
//   forward      out[p][n] = b[n] + sum_{t,k} x[p + s_t][k] W[t][n][k]
//                (one wave = 32 points x 32 output channels, K = 27 taps x 32)
//   input grad   the same kernel with the taps flipped and the channel roles
//                swapped, the ReLU mask of the layer's output applied on load
//   weight grad  dW[t][n][k] = sum_p dz[p][n] x[p + s_t][k] (K = points), the
//                operands staged in LDS point-contiguous, one FP32 partial per
//                block and a fixed-order sum over blocks (deterministic)
// Pointwise layers, pooling, the loss and Adam are plain FP32 kernels.  Master
// weights, gradients and Adam moments are FP32 in the parameter order
// [in.w, in.b, enc0.0.w, enc0.0.b, ..., out.w, out.b] with conv weights
// [C_out][C_in][3][3][3]; the BF16 copies the MFMA kernels read are refreshed
// from the masters after every update.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/arche_net.h"
#include "common.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int NC = 32;           // width
constexpr int LEVELS = 4;
constexpr int NCONV = 14;        // 3x3x3 convolutions
constexpr int WT = 27 * NC * NC;  // weights of one 3x3x3 convolution
constexpr int CONV_PARAMS = WT + NC;
constexpr int64_t P_IN_W = 0, P_IN_B = 64, P_CONV0 = 96;
constexpr int64_t P_OUT_W = P_CONV0 + (int64_t)NCONV * CONV_PARAMS;
constexpr int64_t P_OUT_B = P_OUT_W + NC;
constexpr int64_t NPARAM = P_OUT_B + 1;  // 387,649
constexpr int WG_BLOCKS_MAX = 256;       // weight-gradient partials
constexpr int RED_BLOCKS = 256;          // pointwise-layer partials

struct Geo {
  int D, H, W;
  int64_t P;
};

__device__ inline int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ inline float bf(bf16 x) { return (float)x; }

// ---------------------------------------------------------------------------
// 3x3x3 periodic convolution, 32 -> 32 channels, on MFMA.
// Bw: [27][32 n][32 k] BF16.  MASK: the A operand is x * (y > 0) (input grad of
// a ReLU layer whose output is y).  Writes act(out) as BF16.
template <bool MASK, bool RELU>
__global__ void __launch_bounds__(256)
k_conv3(const bf16* __restrict__ x, const bf16* __restrict__ y, const bf16* __restrict__ Bw,
        const float* __restrict__ bias, bf16* __restrict__ out, Geo g) {
  __shared__ bf16x8 wl[27 * NC * 4];  // [t][n][k/8]
  for (int i = threadIdx.x; i < 27 * NC * 4; i += blockDim.x) wl[i] = ((const bf16x8*)Bw)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, hf = lane >> 5;
  const int64_t ntiles = g.P / 32;
  float bn = bias ? bias[r] : 0.0f;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t p = tile * 32 + r;  // this lane's A row
    const int w = (int)(p % g.W);
    const int h = (int)((p / g.W) % g.H);
    const int d = (int)(p / ((int64_t)g.W * g.H));
    f32x16 acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
      const int dd = wrapi(d + a - 1, g.D);
      for (int c = 0; c < 3; ++c) {
        const int64_t rowbase = ((int64_t)dd * g.H + wrapi(h + c - 1, g.H)) * g.W;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int t = a * 9 + c * 3 + e;
          const int64_t q = (rowbase + wrapi(w + e - 1, g.W)) * NC;
          const bf16x8* src = (const bf16x8*)(x + q);
          bf16x8 a0 = src[hf], a1 = src[2 + hf];
          if (MASK) {
            const bf16x8* ys = (const bf16x8*)(y + q);
            const bf16x8 y0 = ys[hf], y1 = ys[2 + hf];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              if (!(bf(y0[j]) > 0.0f)) a0[j] = (bf16)0.0f;
              if (!(bf(y1[j]) > 0.0f)) a1[j] = (bf16)0.0f;
            }
          }
          const bf16x8 b0 = wl[(t * NC + r) * 4 + hf], b1 = wl[(t * NC + r) * 4 + 2 + hf];
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc, 0, 0, 0);
        }
      }
    }
    // D layout: lane holds column n = r, rows 8*(v/4) + 4*hf + v%4
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 8 * (v / 4) + 4 * hf + (v % 4);
      float o = acc[v] + bn;
      if (RELU) o = fmaxf(o, 0.0f);
      out[(tile * 32 + row) * NC + r] = (bf16)o;
    }
  }
}

// Weight and bias gradient of a 3x3x3 convolution over a range of 32-point
// chunks per block.  dz = dy * (y > 0).  LDS holds, per chunk, dz transposed
// [n][point] and the 27 shifted inputs transposed [t][k][point], so every MFMA
// operand is 8 point-contiguous values.  part: [nblk][27*32*32 + 32] FP32.
__global__ void __launch_bounds__(256)
k_conv3_wgrad(const bf16* __restrict__ x, const bf16* __restrict__ dy, const bf16* __restrict__ y,
              float* __restrict__ part, Geo g) {
  __shared__ __attribute__((aligned(16))) bf16 xs[27 * NC * 32];  // [t][k][pt]
  __shared__ __attribute__((aligned(16))) bf16 zs[NC * 32];       // [n][pt]
  __shared__ float bsum[4][NC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, hf = lane >> 5;
  const int64_t nchunk = g.P / 32;
  f32x16 acc[7];
  for (int i = 0; i < 7; ++i)
    for (int v = 0; v < 16; ++v) acc[i][v] = 0.0f;
  float bacc = 0.0f;  // bias grad, thread < 128 owns (point group, channel chunk)
  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t p0 = ch * 32;
    __syncthreads();  // previous chunk's MFMAs are done with LDS
    // dz: 32 points x 4 chunks of 8 channels
    if (threadIdx.x < 128) {
      const int pt = threadIdx.x >> 2, k8 = threadIdx.x & 3;
      const int64_t q = (p0 + pt) * NC + 8 * k8;
      bf16x8 v = *(const bf16x8*)(dy + q);
      const bf16x8 m = *(const bf16x8*)(y + q);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (!(bf(m[j]) > 0.0f)) v[j] = (bf16)0.0f;
        zs[(8 * k8 + j) * 32 + pt] = v[j];
      }
    }
    // shifted inputs: 27 taps x 32 points x 4 channel chunks
    for (int task = threadIdx.x; task < 27 * 32 * 4; task += blockDim.x) {
      const int t = task / 128, rem = task - t * 128;
      const int pt = rem >> 2, k8 = rem & 3;
      const int64_t p = p0 + pt;
      const int w = (int)(p % g.W);
      const int h = (int)((p / g.W) % g.H);
      const int d = (int)(p / ((int64_t)g.W * g.H));
      const int a = t / 9, c = (t / 3) % 3, e = t % 3;
      const int64_t q = ((((int64_t)wrapi(d + a - 1, g.D) * g.H) + wrapi(h + c - 1, g.H)) * g.W +
                         wrapi(w + e - 1, g.W)) * NC + 8 * k8;
      const bf16x8 v = *(const bf16x8*)(x + q);
#pragma unroll
      for (int j = 0; j < 8; ++j) xs[(t * NC + 8 * k8 + j) * 32 + pt] = v[j];
    }
    __syncthreads();
    if (threadIdx.x < 128) {
      // bias grad: thread (pt group of 8, channel n = threadIdx.x & 31)
      const int n = threadIdx.x & 31, grp = threadIdx.x >> 5;
      float s = 0.0f;
      for (int j = 0; j < 8; ++j) s += bf(zs[n * 32 + 8 * grp + j]);
      bacc += s;
    }
    // MFMA: M = n, N = k, K = points (two steps of 16)
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const int t = wave + 4 * i;
      if (t < 27) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const bf16x8 av = *(const bf16x8*)(zs + r * 32 + 16 * ks + 8 * hf);
          const bf16x8 bv = *(const bf16x8*)(xs + (t * NC + r) * 32 + 16 * ks + 8 * hf);
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i], 0, 0, 0);
        }
      }
    }
  }
  float* dst = part + (size_t)blockIdx.x * (WT + NC);
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const int t = wave + 4 * i;
    if (t < 27) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int n = 8 * (v / 4) + 4 * hf + (v % 4);
        dst[(t * NC + n) * NC + r] = acc[i][v];  // [t][n][k]
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 128) bsum[threadIdx.x >> 5][threadIdx.x & 31] = bacc;
  __syncthreads();
  if (threadIdx.x < NC) dst[WT + threadIdx.x] = ((bsum[0][threadIdx.x] + bsum[1][threadIdx.x]) + bsum[2][threadIdx.x]) +
                                                bsum[3][threadIdx.x];
}

// Sum the partials in block order; write the grads in parameter order
// (W[n][k][t], then the bias) at gdst.
__global__ void __launch_bounds__(256) k_wgrad_finish(const float* __restrict__ part, int nblk, float* __restrict__ gdst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= WT + NC) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * (WT + NC) + i];
  if (i < WT) {
    const int t = i / (NC * NC), n = (i / NC) % NC, k = i % NC;
    gdst[(n * NC + k) * 27 + t] = s;
  } else {
    gdst[i] = s;
  }
}

// BF16 copies of one convolution's weights: forward [t][n][k] = W[n][k][t] and
// input-grad [t][k][n] = W[n][k][26 - t] (flipped taps, swapped channels).
__global__ void __launch_bounds__(256) k_conv_weights(const float* __restrict__ Wm, bf16* __restrict__ fwd,
                                                    bf16* __restrict__ bwd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= WT) return;
  const int t = i / (NC * NC), n = (i / NC) % NC, k = i % NC;
  fwd[i] = (bf16)Wm[(n * NC + k) * 27 + t];        // i = (t, n, k)
  bwd[i] = (bf16)Wm[(k * NC + n) * 27 + (26 - t)];  // i = (t, n=in channel, k=out channel)
}

// ---------------------------------------------------------------------------
// Pointwise layers.
// in: a = g/n0 - 1, b = p/n0 - 1; h = relu(W_in [a b] + b_in)  (BF16 out)
__global__ void __launch_bounds__(256)
k_in_fwd(const double* __restrict__ guess, const double* __restrict__ prev, double n0, const float* __restrict__ prm,
         float* __restrict__ xin, bf16* __restrict__ h, int64_t P) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const float a = (float)(guess[p] / n0 - 1.0), b = (float)(prev[p] / n0 - 1.0);
    xin[2 * p] = a;
    xin[2 * p + 1] = b;
    bf16x8 o[4];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const float z = prm[P_IN_B + c] + prm[P_IN_W + 2 * c] * a + prm[P_IN_W + 2 * c + 1] * b;
      o[c / 8][c % 8] = (bf16)fmaxf(z, 0.0f);
    }
    bf16x8* dst = (bf16x8*)(h + p * NC);
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[j] = o[j];
  }
}

// grads of in.w, in.b from dh and h (mask): per-block partials [nblk][96]
__global__ void __launch_bounds__(256)
k_in_bwd(const float* __restrict__ xin, const bf16* __restrict__ h, const bf16* __restrict__ dh, float* __restrict__ part,
         int64_t P) {
  __shared__ float sh[256];
  const int c = threadIdx.x & 31, lanegrp = threadIdx.x >> 5;  // 8 points in flight per block
  float gw0 = 0.0f, gw1 = 0.0f, gb = 0.0f;
  for (int64_t p = (int64_t)blockIdx.x * 8 + lanegrp; p < P; p += (int64_t)gridDim.x * 8) {
    const float m = bf(h[p * NC + c]) > 0.0f ? 1.0f : 0.0f;
    const float dz = m * bf(dh[p * NC + c]);
    gw0 += dz * xin[2 * p];
    gw1 += dz * xin[2 * p + 1];
    gb += dz;
  }
  float vals[3] = {gw0, gw1, gb};
  for (int q = 0; q < 3; ++q) {
    sh[threadIdx.x] = vals[q];
    __syncthreads();
    if (threadIdx.x < 32) {
      float s = 0.0f;
      for (int j = 0; j < 8; ++j) s += sh[j * 32 + threadIdx.x];
      // layout: in.w [c][2] then in.b [c]
      if (q < 2) part[(size_t)blockIdx.x * 96 + 2 * threadIdx.x + q] = s;
      else part[(size_t)blockIdx.x * 96 + 64 + threadIdx.x] = s;
    }
    __syncthreads();
  }
}

// out: r = W_out h + b_out (FP32); with a target (r* = conv/n0 - 1 - b), the
// loss terms and dr -> dh, partial sums of the loss and of the out.w/out.b
// grads: part [nblk][34]
__global__ void __launch_bounds__(256)
k_out(const bf16* __restrict__ h, const float* __restrict__ prm, const double* __restrict__ guess,
      const double* __restrict__ prev,
      const double* __restrict__ conv, double n0, double* __restrict__ r_out, bf16* __restrict__ dh,
      float* __restrict__ part, int64_t P) {
  __shared__ float sh[34][8];
  float acc[34];
  for (int q = 0; q < 34; ++q) acc[q] = 0.0f;
  float w[NC];
  for (int c = 0; c < NC; ++c) w[c] = prm[P_OUT_W + c];
  const float b = prm[P_OUT_B];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const bf16x8* src = (const bf16x8*)(h + p * NC);
    float hv[NC];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x8 v = src[j];
#pragma unroll
      for (int i = 0; i < 8; ++i) hv[8 * j + i] = bf(v[i]);
    }
    float r = b;
#pragma unroll
    for (int c = 0; c < NC; ++c) r += w[c] * hv[c];
    if (r_out) r_out[p] = r;
    if (conv) {
      const double b = prev[p] / n0 - 1.0;
      const double tgt = conv[p] / n0 - 1.0 - b;
      const float diff = (float)((double)r - tgt);
      const float dr = 2.0f * diff / (float)P;
      acc[33] += diff * diff;
      acc[32] += dr;
      bf16x8 o[4];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        acc[c] += dr * hv[c];
        o[c / 8][c % 8] = (bf16)(dr * w[c]);
      }
      bf16x8* dst = (bf16x8*)(dh + p * NC);
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j] = o[j];
    }
  }
  if (!conv) return;
  // block reduction in a fixed order: lanes of a wave, then waves
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = 0; q < 34; ++q) {
    float v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[q][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 34) {
    float s = 0.0f;
    for (int j = 0; j < 4; ++j) s += sh[threadIdx.x][j];
    part[(size_t)blockIdx.x * 34 + threadIdx.x] = s;
  }
}

// sum per-block partials [nblk][n] in block order into dst[n]
__global__ void __launch_bounds__(256) k_sum_parts(const float* __restrict__ part, int nblk, int n, float* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * n + i];
  dst[i] = s;
}

// mean over 2x2x2 blocks: fine g (D,H,W) -> coarse (D/2,H/2,W/2)
__global__ void __launch_bounds__(256) k_pool(const bf16* __restrict__ in, bf16* __restrict__ out, Geo g) {
  const int64_t Pc = g.P / 8;
  const int Wc = g.W / 2, Hc = g.H / 2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Pc * 4; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = i >> 2;
    const int k8 = (int)(i & 3);
    const int w = (int)(q % Wc), h = (int)((q / Wc) % Hc), d = (int)(q / ((int64_t)Wc * Hc));
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c)
        for (int e = 0; e < 2; ++e) {
          const int64_t p = (((int64_t)(2 * d + a) * g.H) + 2 * h + c) * g.W + 2 * w + e;
          const bf16x8 v = *(const bf16x8*)(in + p * NC + 8 * k8);
#pragma unroll
          for (int j = 0; j < 8; ++j) s[j] += bf(v[j]);
        }
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (bf16)(0.125f * s[j]);
    *(bf16x8*)(out + q * NC + 8 * k8) = o;
  }
}

// fine (D,H,W) grad of pool: d_fine += d_coarse[parent] / 8
__global__ void __launch_bounds__(256) k_pool_bwd_add(const bf16* __restrict__ dc, bf16* __restrict__ df, Geo g) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.P * 4; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i >> 2;
    const int k8 = (int)(i & 3);
    const int w = (int)(p % g.W), h = (int)((p / g.W) % g.H), d = (int)(p / ((int64_t)g.W * g.H));
    const int64_t q = (((int64_t)(d / 2) * (g.H / 2)) + h / 2) * (g.W / 2) + w / 2;
    const bf16x8 c = *(const bf16x8*)(dc + q * NC + 8 * k8);
    bf16x8 f = *(const bf16x8*)(df + p * NC + 8 * k8);
#pragma unroll
    for (int j = 0; j < 8; ++j) f[j] = (bf16)(bf(f[j]) + 0.125f * bf(c[j]));
    *(bf16x8*)(df + p * NC + 8 * k8) = f;
  }
}

// out (fine g) = coarse[parent] + skip
__global__ void __launch_bounds__(256)
k_up_add(const bf16* __restrict__ coarse, const bf16* __restrict__ skip, bf16* __restrict__ out, Geo g) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.P * 4; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = i >> 2;
    const int k8 = (int)(i & 3);
    const int w = (int)(p % g.W), h = (int)((p / g.W) % g.H), d = (int)(p / ((int64_t)g.W * g.H));
    const int64_t q = (((int64_t)(d / 2) * (g.H / 2)) + h / 2) * (g.W / 2) + w / 2;
    const bf16x8 c = *(const bf16x8*)(coarse + q * NC + 8 * k8);
    const bf16x8 s = *(const bf16x8*)(skip + p * NC + 8 * k8);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (bf16)(bf(c[j]) + bf(s[j]));
    *(bf16x8*)(out + p * NC + 8 * k8) = o;
  }
}

// coarse grad of up: sum of the 8 children of d_out (fine g)
__global__ void __launch_bounds__(256) k_up_bwd(const bf16* __restrict__ dout, bf16* __restrict__ dc, Geo g) {
  const int64_t Pc = g.P / 8;
  const int Wc = g.W / 2, Hc = g.H / 2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Pc * 4; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = i >> 2;
    const int k8 = (int)(i & 3);
    const int w = (int)(q % Wc), h = (int)((q / Wc) % Hc), d = (int)(q / ((int64_t)Wc * Hc));
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c)
        for (int e = 0; e < 2; ++e) {
          const int64_t p = (((int64_t)(2 * d + a) * g.H) + 2 * h + c) * g.W + 2 * w + e;
          const bf16x8 v = *(const bf16x8*)(dout + p * NC + 8 * k8);
#pragma unroll
          for (int j = 0; j < 8; ++j) s[j] += bf(v[j]);
        }
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (bf16)s[j];
    *(bf16x8*)(dc + q * NC + 8 * k8) = o;
  }
}

// Adam on FP32 masters (bias-corrected moments)
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ prm, const float* __restrict__ grad, float* __restrict__ m, float* __restrict__ v, int64_t n,
       float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// proposal n = n0 (1 + b + r) = p + n0 r: the previous converged density p
// moved by the learned change, kept at or above PROPOSAL_FLOOR p
constexpr double PROPOSAL_FLOOR = 0.1;
__global__ void __launch_bounds__(256)
k_propose(const double* __restrict__ prev, const double* __restrict__ r, double n0, double* __restrict__ n, int64_t P) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const double rp = r[p], pp = prev[p];
    n[p] = rp == rp ? fmax(pp + n0 * rp, PROPOSAL_FLOOR * pp) : rp;  // a NaN stays visible
  }
}

unsigned grid1(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

struct arche_net {
  Geo g[LEVELS];
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  float *prm = nullptr, *grad = nullptr, *mom1 = nullptr, *mom2 = nullptr;
  bf16 *wf = nullptr, *wb = nullptr;  // [14][27*32*32] forward / input-grad BF16 copies
  int64_t adam_t = 0;
  // activations
  float* xin = nullptr;             // [P0][2]
  bf16* h = nullptr;                // conv_in output
  bf16 *ea[LEVELS] = {}, *s[LEVELS] = {}, *pin[LEVELS] = {};  // enc: first conv out, block out, pooled input
  bf16 *u[LEVELS] = {}, *da[LEVELS] = {}, *dout[LEVELS] = {};  // dec: up+skip, first conv out, block out
  // gradient work
  bf16 *gA[LEVELS] = {}, *gB[LEVELS] = {}, *gS[LEVELS] = {};
  double* r = nullptr;  // [P0] network output
  float* part = nullptr;
  int wg_blocks[LEVELS] = {};
};

namespace {

arche_status nerr(arche_net* n, arche_status s, const std::string& m) {
  if (n) n->err = m;
  return s;
}
#define NK(x)                                                                            \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return nerr(net, ARCHE_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

int conv_index(bool enc, int level, int j) {
  // parameter order: enc0.0, enc0.1, ..., enc3.1, dec2.0, dec2.1, dec1.0, ..., dec0.1
  return enc ? 2 * level + j : 2 * LEVELS + 2 * (LEVELS - 2 - level) + j;
}
int64_t conv_off(int ci) { return P_CONV0 + (int64_t)ci * CONV_PARAMS; }

unsigned conv_blocks(const Geo& g) {
  const int64_t tiles = g.P / 32;
  int64_t b = (tiles + 3) / 4;
  return (unsigned)(b > 512 ? 512 : b);
}

hipError_t conv_fwd(arche_net* n, int ci, const bf16* x, bf16* out, const Geo& g) {
  hipLaunchKernelGGL((k_conv3<false, true>), dim3(conv_blocks(g)), dim3(256), 0, n->stream, x, (const bf16*)nullptr,
                     n->wf + (size_t)ci * WT, n->prm + conv_off(ci) + WT, out, g);
  return hipGetLastError();
}
// dx = conv^T(dy * (y > 0))
hipError_t conv_bwd_data(arche_net* n, int ci, const bf16* dy, const bf16* y, bf16* dx, const Geo& g) {
  hipLaunchKernelGGL((k_conv3<true, false>), dim3(conv_blocks(g)), dim3(256), 0, n->stream, dy, y,
                     n->wb + (size_t)ci * WT, (const float*)nullptr, dx, g);
  return hipGetLastError();
}
hipError_t conv_bwd_w(arche_net* n, int ci, const bf16* x, const bf16* dy, const bf16* y, int level) {
  const Geo& g = n->g[level];
  const int nb = n->wg_blocks[level];
  hipLaunchKernelGGL(k_conv3_wgrad, dim3(nb), dim3(256), 0, n->stream, x, dy, y, n->part, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_wgrad_finish, dim3((WT + NC + 255) / 256), dim3(256), 0, n->stream, (const float*)n->part, nb,
                     n->grad + conv_off(ci));
  return hipGetLastError();
}

hipError_t refresh_weights(arche_net* n) {
  for (int ci = 0; ci < NCONV; ++ci) {
    hipLaunchKernelGGL(k_conv_weights, dim3((WT + 255) / 256), dim3(256), 0, n->stream, n->prm + conv_off(ci),
                       n->wf + (size_t)ci * WT, n->wb + (size_t)ci * WT);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

arche_status forward(arche_net* net, const double* guess, const double* prev, double n0) {
  const Geo* g = net->g;
  hipLaunchKernelGGL(k_in_fwd, dim3(grid1(g[0].P)), dim3(256), 0, net->stream, guess, prev, n0, (const float*)net->prm,
                     net->xin, net->h, g[0].P);
  NK(hipGetLastError());
  const bf16* in = net->h;
  for (int l = 0; l < LEVELS; ++l) {
    if (l > 0) {
      hipLaunchKernelGGL(k_pool, dim3(grid1(g[l].P * 4)), dim3(256), 0, net->stream, (const bf16*)net->s[l - 1],
                         net->pin[l], g[l - 1]);
      NK(hipGetLastError());
      in = net->pin[l];
    }
    NK(conv_fwd(net, conv_index(true, l, 0), in, net->ea[l], g[l]));
    NK(conv_fwd(net, conv_index(true, l, 1), net->ea[l], net->s[l], g[l]));
  }
  const bf16* coarse = net->s[LEVELS - 1];
  for (int l = LEVELS - 2; l >= 0; --l) {
    hipLaunchKernelGGL(k_up_add, dim3(grid1(g[l].P * 4)), dim3(256), 0, net->stream, coarse, (const bf16*)net->s[l],
                       net->u[l], g[l]);
    NK(hipGetLastError());
    NK(conv_fwd(net, conv_index(false, l, 0), net->u[l], net->da[l], g[l]));
    NK(conv_fwd(net, conv_index(false, l, 1), net->da[l], net->dout[l], g[l]));
    coarse = net->dout[l];
  }
  return ARCHE_OK;
}

arche_status check_dims(arche_net* net, const int32_t grid[3]) {
  for (int a = 0; a < 3; ++a)
    if (grid[a] < 8 || grid[a] % 8 != 0) return nerr(net, ARCHE_EINVAL, "grid edges must be multiples of 8");
  return ARCHE_OK;
}

}  // namespace

extern "C" {

int64_t arche_net_param_count(void) { return NPARAM; }

arche_status arche_net_create(const int32_t grid[3], void* hip_stream, arche_net** out) {
  if (!out || !grid) return ARCHE_EINVAL;
  *out = nullptr;
  arche_net* net = new (std::nothrow) arche_net();
  if (!net) return ARCHE_ENOMEM;
  if (check_dims(net, grid) != ARCHE_OK) {
    delete net;
    return ARCHE_EINVAL;
  }
  // the coarsest level (1/512 of the points) must hold whole 32-point MFMA tiles
  if (((int64_t)grid[0] * grid[1] * grid[2]) % (32 * 512) != 0) {
    delete net;
    return ARCHE_EINVAL;
  }
  for (int l = 0; l < LEVELS; ++l) {
    net->g[l].D = grid[0] >> l;
    net->g[l].H = grid[1] >> l;
    net->g[l].W = grid[2] >> l;
    net->g[l].P = (int64_t)net->g[l].D * net->g[l].H * net->g[l].W;
    const int64_t nch = net->g[l].P / 32;
    net->wg_blocks[l] = (int)(nch < WG_BLOCKS_MAX ? nch : WG_BLOCKS_MAX);
  }
  if (hip_stream) {
    net->stream = (hipStream_t)hip_stream;
  } else if (hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking) == hipSuccess) {
    net->own_stream = true;
  } else {
    delete net;
    return ARCHE_EHIP;
  }
  bool ok = true;
  auto al = [&](auto** p, size_t n) { ok = ok && hipMalloc((void**)p, n * sizeof(**p)) == hipSuccess; };
  al(&net->prm, NPARAM);
  al(&net->grad, NPARAM);
  al(&net->mom1, NPARAM);
  al(&net->mom2, NPARAM);
  al(&net->wf, (size_t)NCONV * WT);
  al(&net->wb, (size_t)NCONV * WT);
  const int64_t P0 = net->g[0].P;
  al(&net->xin, 2 * P0);
  al(&net->h, P0 * NC);
  al(&net->r, P0);
  for (int l = 0; l < LEVELS; ++l) {
    const size_t n = (size_t)net->g[l].P * NC;
    al(&net->ea[l], n);
    al(&net->s[l], n);
    if (l > 0) al(&net->pin[l], n);
    if (l < LEVELS - 1) {
      al(&net->u[l], n);
      al(&net->da[l], n);
      al(&net->dout[l], n);
    }
    al(&net->gA[l], n);
    al(&net->gB[l], n);
    al(&net->gS[l], n);
  }
  al(&net->part, (size_t)WG_BLOCKS_MAX * (WT + NC) + (size_t)RED_BLOCKS * 128);
  if (!ok) {
    arche_net_free(net);
    return ARCHE_ENOMEM;
  }
  if (hipMemsetAsync(net->mom1, 0, NPARAM * sizeof(float), net->stream) != hipSuccess ||
      hipMemsetAsync(net->mom2, 0, NPARAM * sizeof(float), net->stream) != hipSuccess ||
      hipMemsetAsync(net->prm, 0, NPARAM * sizeof(float), net->stream) != hipSuccess) {
    arche_net_free(net);
    return ARCHE_EHIP;
  }
  *out = net;
  return ARCHE_OK;
}

arche_status arche_net_set_params(arche_net* net, const float* params_host, int64_t n) {
  if (!net || !params_host || n != NPARAM) return nerr(net, ARCHE_EINVAL, "expected arche_net_param_count() floats");
  NK(hipMemcpyAsync(net->prm, params_host, NPARAM * sizeof(float), hipMemcpyHostToDevice, net->stream));
  NK(hipMemsetAsync(net->mom1, 0, NPARAM * sizeof(float), net->stream));
  NK(hipMemsetAsync(net->mom2, 0, NPARAM * sizeof(float), net->stream));
  net->adam_t = 0;
  NK(refresh_weights(net));
  NK(hipStreamSynchronize(net->stream));
  return ARCHE_OK;
}

arche_status arche_net_get_params(arche_net* net, float* params_host, int64_t n) {
  if (!net || !params_host || n != NPARAM) return nerr(net, ARCHE_EINVAL, "expected arche_net_param_count() floats");
  NK(hipMemcpyAsync(params_host, net->prm, NPARAM * sizeof(float), hipMemcpyDeviceToHost, net->stream));
  NK(hipStreamSynchronize(net->stream));
  return ARCHE_OK;
}

arche_status arche_net_get_grads(arche_net* net, float* grads_host, int64_t n) {
  if (!net || !grads_host || n != NPARAM) return nerr(net, ARCHE_EINVAL, "expected arche_net_param_count() floats");
  NK(hipMemcpyAsync(grads_host, net->grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost, net->stream));
  NK(hipStreamSynchronize(net->stream));
  return ARCHE_OK;
}

arche_status arche_net_forward(arche_net* net, const double* guess, const double* prev, double n0, double* r_out) {
  if (!net || !guess || !prev || !(n0 > 0.0)) return nerr(net, ARCHE_EINVAL, "bad argument");
  arche_status s = forward(net, guess, prev, n0);
  if (s != ARCHE_OK) return s;
  const Geo& g = net->g[0];
  hipLaunchKernelGGL(k_out, dim3(RED_BLOCKS), dim3(256), 0, net->stream, (const bf16*)net->dout[0],
                     (const float*)net->prm, (const double*)nullptr, (const double*)nullptr,
                     (const double*)nullptr, n0,
                     r_out ? r_out : net->r, (bf16*)nullptr, net->part, g.P);
  NK(hipGetLastError());
  return ARCHE_OK;
}

arche_status arche_net_propose(arche_net* net, const double* guess, const double* prev, double n0, double* n_out) {
  if (!n_out) return nerr(net, ARCHE_EINVAL, "bad argument");
  arche_status s = arche_net_forward(net, guess, prev, n0, net ? net->r : nullptr);
  if (s != ARCHE_OK) return s;
  hipLaunchKernelGGL(k_propose, dim3(grid1(net->g[0].P)), dim3(256), 0, net->stream, prev, (const double*)net->r, n0,
                     n_out, net->g[0].P);
  NK(hipGetLastError());
  return ARCHE_OK;
}

arche_status arche_net_loss_grad(arche_net* net, const double* guess, const double* prev, const double* conv, double n0,
                                 double* loss_out) {
  if (!net || !guess || !prev || !conv || !(n0 > 0.0)) return nerr(net, ARCHE_EINVAL, "bad argument");
  arche_status s = forward(net, guess, prev, n0);
  if (s != ARCHE_OK) return s;
  const Geo* g = net->g;
  // output layer, loss and dL/d dout0
  float* pout = net->part + (size_t)WG_BLOCKS_MAX * (WT + NC);
  hipLaunchKernelGGL(k_out, dim3(RED_BLOCKS), dim3(256), 0, net->stream, (const bf16*)net->dout[0],
                     (const float*)net->prm, guess, prev, conv, n0, net->r, net->gA[0], pout, g[0].P);
  NK(hipGetLastError());
  // out.w grads [0..31], out.b [32], loss sum [33]
  float* small = pout + (size_t)RED_BLOCKS * 34;
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, net->stream, (const float*)pout, RED_BLOCKS, 34, small);
  NK(hipGetLastError());
  NK(hipMemcpyAsync(net->grad + P_OUT_W, small, 33 * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  float hsmall[34];
  NK(hipMemcpyAsync(hsmall, small, 34 * sizeof(float), hipMemcpyDeviceToHost, net->stream));
  // decoder, finest first: grad of dout[l] is in gA[l]
  for (int l = 0; l <= LEVELS - 2; ++l) {
    const int c0 = conv_index(false, l, 0), c1 = conv_index(false, l, 1);
    NK(conv_bwd_w(net, c1, net->da[l], net->gA[l], net->dout[l], l));
    NK(conv_bwd_data(net, c1, net->gA[l], net->dout[l], net->gB[l], g[l]));
    NK(conv_bwd_w(net, c0, net->u[l], net->gB[l], net->da[l], l));
    // grad of u[l] -> gS[l] (skip grad, also the input of up)
    NK(conv_bwd_data(net, c0, net->gB[l], net->da[l], net->gS[l], g[l]));
    // coarse grad: sum over children -> grad of dout[l+1] (or of s[top])
    hipLaunchKernelGGL(k_up_bwd, dim3(grid1(g[l + 1].P * 4)), dim3(256), 0, net->stream, (const bf16*)net->gS[l],
                       net->gA[l + 1], g[l]);
    NK(hipGetLastError());
  }
  // encoder, coarsest first: gA[l] holds the grad of s[l] (complete for the top
  // level; the others add their skip grad gS[l] below)
  for (int l = LEVELS - 1; l >= 0; --l) {
    bf16* ds = l == LEVELS - 1 ? net->gA[l] : net->gS[l];
    const int c0 = conv_index(true, l, 0), c1 = conv_index(true, l, 1);
    const bf16* in = l == 0 ? net->h : net->pin[l];
    NK(conv_bwd_w(net, c1, net->ea[l], ds, net->s[l], l));
    NK(conv_bwd_data(net, c1, ds, net->s[l], net->gB[l], g[l]));
    NK(conv_bwd_w(net, c0, in, net->gB[l], net->ea[l], l));
    NK(conv_bwd_data(net, c0, net->gB[l], net->ea[l], net->gA[l], g[l]));  // grad of the block input
    if (l > 0) {
      // pooled input: d s[l-1] += pool^T(grad)
      hipLaunchKernelGGL(k_pool_bwd_add, dim3(grid1(g[l - 1].P * 4)), dim3(256), 0, net->stream,
                         (const bf16*)net->gA[l], net->gS[l - 1], g[l - 1]);
      NK(hipGetLastError());
    }
  }
  // input layer
  hipLaunchKernelGGL(k_in_bwd, dim3(RED_BLOCKS), dim3(256), 0, net->stream, (const float*)net->xin,
                     (const bf16*)net->h, (const bf16*)net->gA[0], pout, g[0].P);
  NK(hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, net->stream, (const float*)pout, RED_BLOCKS, 96,
                     net->grad + P_IN_W);
  NK(hipGetLastError());
  NK(hipStreamSynchronize(net->stream));
  if (loss_out) *loss_out = (double)hsmall[33] / (double)g[0].P;
  return ARCHE_OK;
}

arche_status arche_net_adam_step(arche_net* net, double lr, double beta1, double beta2, double eps) {
  if (!net || !(lr > 0.0)) return nerr(net, ARCHE_EINVAL, "bad argument");
  net->adam_t++;
  const float c1 = (float)(1.0 - std::pow(beta1, (double)net->adam_t));
  const float c2 = (float)(1.0 - std::pow(beta2, (double)net->adam_t));
  hipLaunchKernelGGL(k_adam, dim3(grid1(NPARAM)), dim3(256), 0, net->stream, net->prm, (const float*)net->grad,
                     net->mom1, net->mom2, NPARAM, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
  NK(hipGetLastError());
  NK(refresh_weights(net));
  return ARCHE_OK;
}

arche_status arche_net_debug_get(arche_net* net, int32_t which, int32_t level, float* host) {
  if (!net || !host || level < 0 || level >= LEVELS) return nerr(net, ARCHE_EINVAL, "bad argument");
  bf16* t[10] = {level == 0 ? net->h : nullptr, net->ea[level], net->s[level], net->pin[level], net->u[level],
                 net->da[level], net->dout[level], net->gA[level], net->gB[level], net->gS[level]};
  if (which < 0 || which >= 10 || !t[which]) return nerr(net, ARCHE_EINVAL, "no such tensor");
  const size_t n = (size_t)net->g[level].P * NC;
  std::vector<bf16> tmp(n);
  NK(hipMemcpyAsync(tmp.data(), t[which], n * sizeof(bf16), hipMemcpyDeviceToHost, net->stream));
  NK(hipStreamSynchronize(net->stream));
  for (size_t i = 0; i < n; ++i) host[i] = (float)tmp[i];
  return ARCHE_OK;
}

arche_status arche_net_sync(arche_net* net) {
  if (!net) return ARCHE_EINVAL;
  NK(hipStreamSynchronize(net->stream));
  return ARCHE_OK;
}

const char* arche_net_last_error(const arche_net* net) { return net ? net->err.c_str() : ""; }

void arche_net_free(arche_net* net) {
  if (!net) return;
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  void* ptrs[] = {net->prm, net->grad, net->mom1, net->mom2, net->wf, net->wb, net->xin, net->h, net->r, net->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int l = 0; l < LEVELS; ++l) {
    void* q[] = {net->ea[l], net->s[l], net->pin[l], net->u[l], net->da[l], net->dout[l], net->gA[l], net->gB[l],
                 net->gS[l]};
    for (void* p : q)
      if (p) (void)hipFree(p);
  }
  if (net->own_stream) (void)hipStreamDestroy(net->stream);
  delete net;
}

}  // extern "C"
