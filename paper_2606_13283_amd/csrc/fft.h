// FP64 3D real<->complex FFT for gfx950 on C-ordered [Nx][Ny][Nz] real fields and
// [Nx][Ny][Nz/2+1] half spectra (the periodic grid of the paper's Sec. 2.3).
//
// Three passes per transform.  The z pass packs two neighbouring real rows into one
// complex line (real + i*imag), transforms it in LDS and splits the result by
// Hermitian symmetry; the y and x passes transform tiles of [L][TK] complex values
// (TK neighbouring k_z columns per line, so every global access is a contiguous
// run of TK*16 bytes).  Each line is a mixed-radix (2, 3, 4, 5) Stockham transform
// ping-ponging between two LDS buffers.  Transforms are unnormalised; callers pass
// a scale applied on the last write.
#pragma once

#include "common.h"

struct FftAxis {
  int L;
  int nst;
  int radix[8];
  cplx* tw;  // device, L entries exp(-2 pi i m / L)
};

struct FftPlan {
  int N[3];
  int Nh;        // Nz/2 + 1
  int64_t ng;    // Nx*Ny*Nz
  int64_t nh;    // Nx*Ny*Nh
  FftAxis ax[3];
  bool ok;
};

// Returns false (and leaves plan->ok false) if a size is odd, > 1024 or has a
// prime factor other than 2, 3, 5.
bool fft_plan_create(FftPlan* plan, const int N[3]);
// the same with the twiddle tables from a caller's allocator (released by
// fft_plan_destroy_with through `release`)
bool fft_plan_create_with(FftPlan* plan, const int N[3], void* (*alloc)(size_t, void*),
                          void (*release)(void*, void*), void* stream);
void fft_plan_destroy_with(FftPlan* plan, void (*release)(void*, void*), void* stream);
// Fills sizes and radix plans only (no allocation, tw left null): the caller
// points each axis's tw at L twiddles it provides (fft_twiddles_host's values).
bool fft_plan_describe(FftPlan* plan, const int N[3]);
// exp(-2 pi i m / L), m = 0..L-1, rounded from long double
void fft_twiddles_host(int L, cplx* tw);
void fft_plan_destroy(FftPlan* plan);
bool fft_size_supported(int n);

// Work fused into the first pass of a real-to-complex transform (R2C) or into the
// last pass of a complex-to-real one (C2R), and the spectral work fused into the
// x pass (the last pass of R2C, the first of C2R).  Used by the SCF iteration;
// sizes without a compile-time plan run the unfused sequence instead.
enum {
  FUSE_NONE = 0,
  R2C_IN_SQRT = 1,      // transform sqrt(in)
  R2C_IN_MIX_SQRT = 2,  // n_o = in + w (n_i - in); n_i <- n_o; transform sqrt(n_o)
  R2C_OUT_LAP = 1,      // out <- -(2 pi |k|)^2 out
  R2C_OUT_UH = 2,       // out stored; partial sums of w_k |nhat_i - out|^2 / (pi k^2), k != 0
  C2R_IN_MIX = 1,       // n_o^ = in + w (nhat_i - in); nhat_i <- n_o^; transform n_o^ / (pi k^2)
  C2R_OUT_UVW = 1       // no store; partial sums of (v_vW[n_i] - v_vW[n_a]) (n_i - n_a), v = -(lam/2) out/sqrt(n)
};
struct FftFuse {
  const double* w;       // mixing weight (device scalar)
  double* n_i;           // R2C_IN_MIX_SQRT, C2R_OUT_UVW
  const double* n_a;     // C2R_OUT_UVW
  const double* lap_i;   // C2R_OUT_UVW
  const double* uvw_w;   // C2R_OUT_UVW: (n_i - n_a)/sqrt(n_a) from the SCF kernel, which has summed the
                         // v_vW[n_i] part of U_vW (null: the pass forms all of U_vW from n_i, n_a, lap_i)
  cplx* nhat_i;          // R2C_OUT_UH (read), C2R_IN_MIX (read/write)
  double* partials;      // one double per block of the fused pass
  double lam;            // C2R_OUT_UVW
  double L[3];           // cell edges, for |k|
  const int* stop;       // device flag: when nonzero the pass does nothing (null: always run)
};
// k-vector helpers of the x pass: element k of column `line` in the tile at outer
// index o (the y index) is the point (m_x = k, m_y = o, m_z = c0 + line).
// x passes tile the whole (y, k_z) plane of an x index as one run of N_y N_h
// columns (col = m_y N_h + m_z), so that a tile of TK columns is one contiguous
// 16 TK-byte run of every x plane, aligned as the plane is.
struct XGeom {
  int Nx, Ny, Nz;
  double Lx, Ly, Lz;
  __device__ double k2(int mx, int my, int mz) const {
    const double kx = (double)(mx <= Nx / 2 ? mx : mx - Nx) / Lx;
    const double ky = (double)(my <= Ny / 2 ? my : my - Ny) / Ly;
    const double kz = (double)mz / Lz;
    return kx * kx + ky * ky + kz * kz;
  }
  // |k|^2 at x index mx and plane column col
  __device__ double k2c(int mx, int col) const {
    const int nh = Nz / 2 + 1;
    const int my = col / nh;
    return k2(mx, my, col - my * nh);
  }
  __device__ double weight(int mz) const { return (mz == 0 || 2 * mz == Nz) ? 1.0 : 2.0; }
  __device__ double weightc(int col) const { return weight(col % (Nz / 2 + 1)); }
};

// Arguments of one strided pass (lines along y or x of the half spectrum).
struct StridedArgs {
  cplx* data;        // transformed in place (MODE 3: the work array)
  const cplx* src;   // MODE 3: the input spectrum
  const cplx* tw;    // [L] exp(-2 pi i m / L)
  int64_t es, os;    // element stride along the line, stride between outer indices
  int ncols, nchunk; // columns per outer index (y passes: k_z values; x passes: the
                     // whole (y, k_z) plane, one outer index), tiles of TK columns
  double scale;
  FftFuse f;
  XGeom g;
};

// Arguments of one z pass: rows of the real field paired into complex lines.
struct ZArgs {
  const void* in;    // R2C: real [ng]; C2R: half spectrum [nh]
  void* out;         // R2C: half spectrum; C2R: real field
  const cplx* tw;    // [L]
  int64_t npairs;    // Nx*Ny/2
  double in_scale, out_scale;
  FftFuse f;
};

// One pass of a compile-time transform: what a single-grid launch takes, and the
// job a batched launch runs for one grid.
// FFT_PASS_ZY_R2C / FFT_PASS_YZ_C2R: the z and y passes of a grid with N_y = N_z
// fused into one pass over x planes held in LDS (ZArgs; one block per plane);
// FFT_PASS_NOP: the slot the fused pass frees (launches nothing).
enum {
  FFT_PASS_STRIDED = 0,
  FFT_PASS_Z_R2C = 1,
  FFT_PASS_Z_C2R = 2,
  FFT_PASS_ZY_R2C = 3,
  FFT_PASS_YZ_C2R = 4,
  FFT_PASS_NOP = 5
};
struct FftPass {
  int kind;        // FFT_PASS_*
  int L;           // line length
  int sign, mode;  // strided: transform sign and MODE; z passes: FIN or FOUT code
  int var;         // tile variant (fft_tune)
  unsigned nblocks;
  StridedArgs s;   // FFT_PASS_STRIDED
  ZArgs z;         // the z passes
};
// The three passes of a fused transform (fft_r2c_fused / fft_c2r_fused with the
// same arguments); false if the plan has no compile-time kernels.  With plane
// passes (fft_plane_fusable) the z and y passes are one and the other slot is a
// FFT_PASS_NOP.
bool fft_r2c_passes(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale, int fin, int fout,
                    const FftFuse& f, FftPass out3[3]);
bool fft_c2r_passes(const FftPlan* p, const cplx* in, cplx* work, double* out, double out_scale, int fin, int fout,
                    const FftFuse& f, FftPass out3[3]);
hipError_t fft_pass_launch(const FftPass& ps, hipStream_t s);
// Two independent passes in one launch (the blocks of a, then those of b) where a
// combined kernel exists, else one after the other.
hipError_t fft_dual_launch(const FftPass& a, const FftPass& b, hipStream_t s);

// Tile autotuner: for each line length of the plan outside the batched set,
// time the tile variants of the y, x and z passes on the scratch arrays (any
// contents) and keep the fastest for the rest of the process (the first plan of
// a length decides; later plans reuse it).  A variant changes which block sums
// which terms of the fused partial sums, so results agree to rounding across
// variants and are reproducible for a fixed choice.  ARCHE_FFT_TUNE=0 in the
// environment keeps the default tiles.
hipError_t fft_tune(const FftPlan* p, cplx* scratch_c, double* scratch_r, hipStream_t s);
// the variant in use for (pass 0 y / 1 x / 2 z, line length); force >= 0 sets it
int fft_tile_variant(int pass, int L, int force);

// Batched passes (fft_batch.hip): one launch runs the jobs[j] (device array of
// FftPass, all of the same kind, sign and mode, line lengths within
// fft_batch_supported) with job j owning blocks [bbeg[j], bbeg[j+1]).
bool fft_batch_supported(int L);
hipError_t fft_batch_launch(int kind, int sign, int mode, const FftPass* jobs, const int* bbeg, int njobs,
                            unsigned nblocks, hipStream_t s);

bool fft_fusable(const FftPlan* p);
// x passes of line length L have the MODE 4 round trip (forward, Laplacian,
// inverse in one pass)
bool fft_x_roundtrip(int L);
// N_y = N_z with a plane kernel for that length (the plane fits in LDS)
bool fft_plane_fusable(const FftPlan* p);
// blocks of an x pass re-tiled by N_x/2 + 1 columns (its launch beside a plane pass)
int fft_x_blocks_wide(const FftPlan* p);
// number of blocks (= partial sums) of the fused x pass and of the fused z pass
int fft_x_blocks(const FftPlan* p);
int fft_z_blocks(const FftPlan* p);
hipError_t fft_r2c_fused(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale, int fin,
                         int fout, const FftFuse& f, hipStream_t s);
hipError_t fft_c2r_fused(const FftPlan* p, const cplx* in, cplx* work, double* out, double out_scale, int fin, int fout,
                         const FftFuse& f, hipStream_t s);

// in: real [ng] (read with `in_scale`), out: complex [nh]; out is multiplied by out_scale.
hipError_t fft_r2c(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale,
                   hipStream_t s);
// in/out: complex [nh] is destroyed (used as work space); out real [ng] times out_scale.
hipError_t fft_c2r(const FftPlan* p, cplx* in, double* out, double out_scale, hipStream_t s);
