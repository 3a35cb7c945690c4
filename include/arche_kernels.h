/*
 * arche_kernels.h -- kernel-level entry points of libarche.so, for callers that
 * hold their own device buffers (and for parity tests of single steps of the
 * path).  Same conventions as arche.h: FP64, C row-major, arche_status returns,
 * no call aborts or prints.  Pointers named d_* are device memory on the current
 * HIP device, owned by the caller; `stream` is a hipStream_t (NULL = default).
 * Complex arrays are interleaved (re, im) doubles.
 */
#ifndef ARCHE_KERNELS_H
#define ARCHE_KERNELS_H

#include "arche.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Unnormalised 3D real-to-complex DFT of the periodic grid of Sec. 2.3:
 * d_out[i][j][k] = sum_r d_in[r] exp(-2 pi i (i x/Nx + j y/Ny + k z/Nz)) for
 * k = 0..Nz/2 (half spectrum [Nx][Ny][Nz/2+1] complex).  grid as in
 * arche_params.grid (EINVAL otherwise).  Blocks until done. */
arche_status arche_k_fft_r2c(const int32_t grid[3], const double *d_in, double *d_out, void *stream);

/* Inverse of the above without the 1/N factor: d_out[r] = sum over the full box of
 * F(m) exp(+2 pi i m.r/N), with F the Hermitian extension of the half spectrum
 * d_in (the imaginary parts of the self-conjugate k_z = 0 and N_z/2 entries do
 * not enter, as for any real field).  d_in is not modified.  Blocks until done. */
arche_status arche_k_fft_c2r(const int32_t grid[3], const double *d_in, double *d_out, void *stream);

/* Largest half spectrum (complex values, Nx*Ny*(Nz/2+1)) that
 * arche_k_fft_c2r_noalloc accepts: that of a 128^3 grid (16.25 MiB of work space in
 * the scratch array, which also holds 342 KiB of twiddle tables). */
#define ARCHE_NOALLOC_MAX_NH 1064960

/* arche_k_fft_c2r for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same transform, the same kernels and the same result, with its work
 * copy of the spectrum and the twiddle tables in a library-owned static device
 * array instead of a per-call hipMalloc.  The caller still owns d_in (not
 * modified) and d_out.  Stream-ordered: it returns once the work is enqueued on
 * `stream` and does not synchronise; d_out is ready when the stream reaches
 * that point.
 *   - EINVAL if grid is not supported (as arche_k_fft_c2r) or
 *     Nx*Ny*(Nz/2+1) > ARCHE_NOALLOC_MAX_NH; nothing is enqueued then.
 *   - The first call on a device sets up that device's copy of the array
 *     (resolves its address, uploads the twiddle tables with one blocking
 *     copy); later calls allocate nothing and do not block.
 *   - The array is shared by every call on the device and keeps the last
 *     call's contents: calls that overlap on one device (other streams, other
 *     host threads without ordering) race on it and must be serialised by the
 *     caller.
 * The array holds one device's copy until the process ends. */
arche_status arche_k_fft_c2r_noalloc(const int32_t grid[3], const double *d_in, double *d_out, void *stream);

/* Complete Fermi-Dirac integrals I_j(x) = int_0^inf t^j/(exp(t-x)+1) dt
 * (Sec. 2.2, with eq. SCF1) for j = -1/2, 1/2, 3/2 at n points d_x; any output
 * may be NULL.  Blocks until done. */
arche_status arche_k_fermi_dirac(int64_t n, const double *d_x, double *d_im12, double *d_ip12, double *d_ip32,
                                 void *stream);

/* I_{1/2}(x) and its first three derivatives in x at n points d_x, as the SCF
 * kernel evaluates them: d_d1 = I_{-1/2}/2 (dI_j/dx = j I_{j-1}), which drives
 * the Newton search of mu (eq. newtonmu); d_d2 and d_d3 build the cubic model of
 * N(mu) that starts that search.  Any output may be NULL.  Blocks until done. */
arche_status arche_k_fermi_dirac_derivs(int64_t n, const double *d_x, double *d_d0, double *d_d1, double *d_d2,
                                        double *d_d3, void *stream);

/* Copies of internal fields of a context after a solve (host destination). */
enum {
  ARCHE_DBG_VIE = 0,    /* V^ie(r) [ng] (Sec. 2.4) */
  ARCHE_DBG_VI = 1,     /* last input potential V_i [ng] */
  ARCHE_DBG_NA = 2,     /* active density n_a [ng] */
  ARCHE_DBG_NI = 3,     /* input density n_i [ng] */
  ARCHE_DBG_SZP = 4,    /* charge structure factor S_Z(k) on the half box [nh] complex */
  ARCHE_DBG_SZM = 5,    /* S_Z at k with its Nyquist components negated [nh] complex */
  ARCHE_DBG_NHAT_A = 6, /* spectrum of n_a, (|Omega|/N_g) DFT, half box [nh] complex */
  ARCHE_DBG_FPP = 7     /* real-space Ewald forces [n_atoms][3] */
};
arche_status arche_debug_get(arche_ctx *ctx, int32_t which, double *dst_host);

/* One-center initial density (Sec. 2.5.1) for ions at pos_host from the last
 * converged step, into n_init_host [ng]; *used_fallback = 1 if it fell back to the
 * uniform density.  ESTATE without a converged previous step.  The context's next
 * solve starts afresh (the guess is not kept as a solved state). */
arche_status arche_debug_one_center(arche_ctx *ctx, const double *pos_host, double *n_init_host,
                                    int32_t *used_fallback);
/* As arche_debug_one_center, and raw_host (may be NULL) [Nx][Ny][Nz] receives
 * the learned proposal's guide G = n0 + the one-center superposition's change
 * from the previous to the new positions (arche_net.h). */
arche_status arche_debug_one_center2(arche_ctx *ctx, const double *pos_host, double *n_init_host,
                                     int32_t *used_fallback, double *raw_host);

/* Per-kernel timing.  When enabled, every launch of the kernels below made by
 * calls on ctx is bracketed by a pair of hipEvents on the context's stream and
 * the elapsed times are summed.  Each event pair costs about 10 us of idle GPU
 * time between launches, so time only the kinds needed: on = 0 disables,
 * on = 1 times every kind, any other value times the kinds whose bit is set in
 * on >> 1 (e.g. 2 << ARCHE_PROF_SCF_ACTIVE for the SCF kernel alone).
 *   ARCHE_PROF_SCF_ACTIVE   the cooperative kernel of one SCF iteration
 *                           (potential, Newton search of mu, active density)
 *   ARCHE_PROF_FFT_Z        the z passes of the 3D FFTs (R2C and C2R)
 *   ARCHE_PROF_FFT_STRIDED  the y and x passes of the 3D FFTs */
enum { ARCHE_PROF_SCF_ACTIVE = 0, ARCHE_PROF_FFT_Z = 1, ARCHE_PROF_FFT_STRIDED = 2 };
arche_status arche_profile_enable(arche_ctx *ctx, int32_t on);
arche_status arche_profile_reset(arche_ctx *ctx);
/* Time one launch in `every` of each kind (1, the default and what
 * arche_profile_enable sets: all of them); the
 * launches count of arche_profile_read counts the timed ones.  Sampling keeps
 * the event pairs' idle time out of the launches that are not timed.  EINVAL
 * for every < 1, ESTATE unless profiling is enabled. */
arche_status arche_profile_sample(arche_ctx *ctx, int32_t every);
/* ESTATE unless profiling is enabled; EINVAL for an unknown kind */
arche_status arche_profile_read(arche_ctx *ctx, int32_t kind, double *total_ms, int64_t *launches);

/* Convergence history of the last arche_scf_solve / arche_md_step solve on ctx
 * (empty after batched solves): *n_rows iterations, each row of 10 doubles
 * [iteration, residual, mixing weight w, mu, K, U = U_H + U_xc + U_vW,
 *  max |n_i - n_a| / n_a, Newton passes, More weight on, error flag], one
 * row per iteration.  rows_host may be NULL to query the count. */
arche_status arche_debug_history(arche_ctx *ctx, double *rows_host, int32_t max_rows, int32_t *n_rows);

/* Contexts alive in the process (arche_scf_init .. arche_scf_free, batch members
 * included).  While it is 1 the SCF kernel runs as a plain launch of its
 * occupancy-sized grid; otherwise as a cooperative launch (both compute the same
 * bits). */
int32_t arche_debug_live_contexts(void);

/* FFT tile variant in use for line length L in pass 0 (y), 1 (x) or 2 (z):
 * 0 = 16 columns (strided) / 32 or 16 row pairs (z) per 256-thread block,
 * 1 = 8 per 128 threads, 2 = 4 per 64 threads (lengths above 96 only).  The
 * first context of a length times the variants and keeps the fastest
 * (ARCHE_FFT_TUNE=0 disables).  force in {0,1,2} sets the variant for contexts
 * created afterwards (force < 0: query only).  Returns the variant, -1 for a
 * bad argument. */
int32_t arche_fft_tile(int32_t pass, int32_t L, int32_t force);

#ifdef __cplusplus
}
#endif

#endif /* ARCHE_KERNELS_H */
