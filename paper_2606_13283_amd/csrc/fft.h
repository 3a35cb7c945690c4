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
  cplx* nhat_i;          // R2C_OUT_UH (read), C2R_IN_MIX (read/write)
  double* partials;      // one double per block of the fused pass
  double lam;            // C2R_OUT_UVW
  double L[3];           // cell edges, for |k|
};
bool fft_fusable(const FftPlan* p);
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
