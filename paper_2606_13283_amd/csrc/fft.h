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

// in: real [ng] (read with `in_scale`), out: complex [nh]; out is multiplied by out_scale.
hipError_t fft_r2c(const FftPlan* p, const double* in, cplx* out, double in_scale, double out_scale,
                   hipStream_t s);
// in/out: complex [nh] is destroyed (used as work space); out real [ng] times out_scale.
hipError_t fft_c2r(const FftPlan* p, cplx* in, double* out, double out_scale, hipStream_t s);
