// Batched compile-time FFT passes: one launch runs one pass for many grids of
// possibly different sizes.  Job j (an FftPass) owns the blocks
// [bbeg[j], bbeg[j+1]); each block finds its job by binary search, then runs
// exactly the tile body the single-grid kernel runs for that block, so every
// grid's result is bit-identical to its own unbatched transform.  LDS is sized
// for the largest line length of the batched set.
#include "fft.h"
#include "fft_bodies.h"

namespace {

using namespace fftct;

#define ARCHE_BATCH_SIZES(X) X(16) X(20) X(24) X(30) X(32) X(40) X(48) X(50) X(54) X(60) X(64) X(72) X(80) X(96)

template <int L>
constexpr int z_lds_need() {
  return z_r2c_lds<L, ct_rows<L>()>();
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kMaxL = 96;
constexpr int kStridedLds = cmax(cmax(strided_lds<96, CT_TK>(), strided_lds<80, CT_TK>()), strided_lds<72, CT_TK>());
constexpr int kZLds = cmax(cmax(cmax(cmax(z_lds_need<96>(), z_lds_need<80>()), cmax(z_lds_need<72>(), z_lds_need<64>())),
                                cmax(cmax(z_lds_need<60>(), z_lds_need<54>()), cmax(z_lds_need<50>(), z_lds_need<48>()))),
                           cmax(cmax(cmax(z_lds_need<40>(), z_lds_need<32>()), cmax(z_lds_need<30>(), z_lds_need<24>())),
                                cmax(z_lds_need<20>(), z_lds_need<16>())));

__device__ inline int find_job(const int* __restrict__ bbeg, int njobs) {
  int lo = 0, hi = njobs - 1;
  const int b = (int)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bbeg[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int S, int MODE>
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_strided_batch(const FftPass* __restrict__ jobs, const int* __restrict__ bbeg, int njobs) {
  const int j = find_job(bbeg, njobs);
  const FftPass& J = jobs[j];
  if (J.s.f.stop && *J.s.f.stop) return;
  __shared__ cplx lds[kStridedLds];
  __shared__ cplx tw[kMaxL];
  __shared__ double sh[ARCHE_BLOCK / 64];
  const unsigned bid = blockIdx.x - (unsigned)bbeg[j];
  switch (J.L) {
#define X(n)                                                          \
  case n:                                                             \
    strided_body<n, CT_TK, S, MODE>(J.s, bid, lds, tw, sh); \
    break;
    ARCHE_BATCH_SIZES(X)
#undef X
    default:
      break;
  }
}

template <int FIN>
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_zr2c_batch(const FftPass* __restrict__ jobs, const int* __restrict__ bbeg, int njobs) {
  const int j = find_job(bbeg, njobs);
  const FftPass& J = jobs[j];
  if (J.z.f.stop && *J.z.f.stop) return;
  __shared__ cplx lds[kZLds];
  __shared__ cplx tw[kMaxL];
  const unsigned bid = blockIdx.x - (unsigned)bbeg[j];
  switch (J.L) {
#define X(n)                                                  \
  case n:                                                     \
    z_r2c_body<n, ct_rows<n>(), FIN>(J.z, bid, lds, tw); \
    break;
    ARCHE_BATCH_SIZES(X)
#undef X
    default:
      break;
  }
}

template <int FOUT>
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_zc2r_batch(const FftPass* __restrict__ jobs, const int* __restrict__ bbeg, int njobs) {
  const int j = find_job(bbeg, njobs);
  const FftPass& J = jobs[j];
  if (J.z.f.stop && *J.z.f.stop) return;
  __shared__ cplx lds[kZLds];
  __shared__ cplx tw[kMaxL];
  __shared__ double sh[ARCHE_BLOCK / 64];
  const unsigned bid = blockIdx.x - (unsigned)bbeg[j];
  switch (J.L) {
#define X(n)                                                       \
  case n:                                                          \
    z_c2r_body<n, ct_rows<n>(), FOUT>(J.z, bid, lds, tw, sh); \
    break;
    ARCHE_BATCH_SIZES(X)
#undef X
    default:
      break;
  }
}

}  // namespace

bool fft_batch_supported(int L) {
  switch (L) {
#define X(n) case n:
    ARCHE_BATCH_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

hipError_t fft_batch_launch(int kind, int sign, int mode, const FftPass* jobs, const int* bbeg, int njobs,
                            unsigned nblocks, hipStream_t s) {
  if (kind == FFT_PASS_NOP) return hipSuccess;
  if (njobs <= 0 || nblocks == 0) return hipSuccess;
  const dim3 grid(nblocks), blk(ARCHE_BLOCK);
  if (kind == FFT_PASS_STRIDED) {
    if (mode == 0 && sign < 0) hipLaunchKernelGGL((k_strided_batch<-1, 0>), grid, blk, 0, s, jobs, bbeg, njobs);
    else if (mode == 0) hipLaunchKernelGGL((k_strided_batch<+1, 0>), grid, blk, 0, s, jobs, bbeg, njobs);
    else if (mode == 1) hipLaunchKernelGGL((k_strided_batch<-1, 1>), grid, blk, 0, s, jobs, bbeg, njobs);
    else if (mode == 2) hipLaunchKernelGGL((k_strided_batch<-1, 2>), grid, blk, 0, s, jobs, bbeg, njobs);
    else hipLaunchKernelGGL((k_strided_batch<+1, 3>), grid, blk, 0, s, jobs, bbeg, njobs);
  } else if (kind == FFT_PASS_Z_R2C) {
    if (mode == 0) hipLaunchKernelGGL((k_zr2c_batch<0>), grid, blk, 0, s, jobs, bbeg, njobs);
    else if (mode == 1) hipLaunchKernelGGL((k_zr2c_batch<1>), grid, blk, 0, s, jobs, bbeg, njobs);
    else hipLaunchKernelGGL((k_zr2c_batch<2>), grid, blk, 0, s, jobs, bbeg, njobs);
  } else {
    if (mode == 0) hipLaunchKernelGGL((k_zc2r_batch<0>), grid, blk, 0, s, jobs, bbeg, njobs);
    else hipLaunchKernelGGL((k_zc2r_batch<1>), grid, blk, 0, s, jobs, bbeg, njobs);
  }
  return hipGetLastError();
}
