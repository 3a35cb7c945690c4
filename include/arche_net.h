/*
 * arche_net.h -- learned initial density for the SCF of arche.h, replacing the
 * one-center guess (Sec. 2.5.1): a 3D U-Net on the periodic grid.  Inputs: the
 * guide G = n0 + the one-center superposition's change between the previous
 * and the new positions, g^ (S_Z(new) - S_Z(old)) in real space, and the
 * previous converged density p.  With a = G/n0 - 1 and b = p/n0 - 1
 * (n0 = N_e/|Omega|) the network returns r, the predicted change n/n0 - 1 - b
 * of the converged density.  In an SCF solve the proposal is
 * n = p + n0 LP(r), LP a low pass exp(-(|k|/k_c)^2) with k_c a quarter of the
 * smallest Nyquist frequency (short-wavelength error in a guess slows the SCF
 * down), kept at or above 0.1 p and renormalised.
 *
 * Network: 1x1x1 input layer 2->32 + ReLU; four levels of width 32, each two
 * periodic 3x3x3 convolutions + ReLU (encoder), 2x2x2 mean pooling between
 * levels; decoder levels 2..0 take nearest-upsampled coarse features plus the
 * encoder's features of that level and apply two 3x3x3 convolutions + ReLU;
 * 1x1x1 output layer 32->1.  387,649 parameters.  Weights and activations are
 * BF16 with FP32 accumulation on the matrix cores; master weights, gradients
 * and Adam moments are FP32.
 *
 * Parameter order (arche_net_set_params / get_params / get_grads, FP32):
 *   in.w [32][2], in.b [32],
 *   enc0.0, enc0.1, enc1.0, enc1.1, enc2.0, enc2.1, enc3.0, enc3.1,
 *   dec2.0, dec2.1, dec1.0, dec1.1, dec0.0, dec0.1  (each .w [32][32][3][3][3] then .b [32]),
 *   out.w [1][32], out.b [1].
 * A 3x3x3 convolution is the cross-correlation
 *   out[o](i,j,k) = b[o] + sum_{c,a,b',e} w[o][c][a][b'][e] x[c](i+a-1, j+b'-1, k+e-1)
 * with indices taken modulo the grid.
 *
 * Device pointers (suffix _dev) are on the net's device; fields are FP64
 * [Nx][Ny][Nz].  Every call returns an arche_status; arche_net_last_error
 * describes a failure.  A net is used by one host thread at a time.
 */
#ifndef ARCHE_NET_H
#define ARCHE_NET_H

#include <stdint.h>

#include "arche.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arche_net arche_net;

int64_t arche_net_param_count(void);

/* A net for grids [Nx][Ny][Nz]: every edge a multiple of 8 and Nx*Ny*Nz a
 * multiple of 16384 (the coarsest level holds whole 32-point tiles), else
 * EINVAL.  Parameters start at zero: call arche_net_set_params.  hip_stream as
 * in arche_scf_init. */
arche_status arche_net_create(const int32_t grid[3], void *hip_stream, arche_net **out);

/* Copy n == arche_net_param_count() FP32 parameters in (resets the Adam
 * moments) or out. */
arche_status arche_net_set_params(arche_net *net, const float *params_host, int64_t n);
arche_status arche_net_get_params(arche_net *net, float *params_host, int64_t n);

/* r_out_dev [Nx][Ny][Nz] FP64 (may be NULL: kept inside the net).  Asynchronous
 * on the net's stream. */
arche_status arche_net_forward(arche_net *net, const double *guess_dev, const double *prev_dev, double n0,
                               double *r_out_dev);

/* n_out_dev = max(prev + n0 r, 0.1 prev) pointwise (no low pass, not
 * renormalised).  Asynchronous. */
arche_status arche_net_propose(arche_net *net, const double *guess_dev, const double *prev_dev, double n0,
                               double *n_out_dev);

/* Loss L = mean over the grid of (r - r*)^2 with r* = conv/n0 - 1 - b, and its
 * gradient with respect to every parameter (kept in the net, replacing the
 * previous one; read with arche_net_get_grads).  Synchronous; *loss_out may be
 * NULL. */
arche_status arche_net_loss_grad(arche_net *net, const double *guess_dev, const double *prev_dev,
                                 const double *conv_dev, double n0, double *loss_out);
arche_status arche_net_get_grads(arche_net *net, float *grads_host, int64_t n);

/* One Adam update of the parameters from the last gradient (bias-corrected
 * moments; the BF16 weight copies are refreshed). */
arche_status arche_net_adam_step(arche_net *net, double lr, double beta1, double beta2, double eps);

/* Debug: copy an internal BF16 tensor [P_level][32] (channels last) to host
 * FP32.  which: 0 input-layer output (level 0 only), 1 first conv of the
 * encoder level, 2 encoder level output, 3 pooled input (level > 0), 4 decoder
 * input up+skip, 5 first decoder conv, 6 decoder level output (levels < 3);
 * 7, 8, 9 gradient work tensors A, B, S of the last arche_net_loss_grad
 * (A: grad of the level's block output / input, B: grad of the first conv's
 * output, S: grad of the skip).  Level l has (Nx/2^l)(Ny/2^l)(Nz/2^l) points. */
arche_status arche_net_debug_get(arche_net *net, int32_t which, int32_t level, float *host);

arche_status arche_net_sync(arche_net *net);
const char *arche_net_last_error(const arche_net *net);
void arche_net_free(arche_net *net);

/* Use `net` (same grid as the context; may be NULL to detach) for solves with
 * p.init == ARCHE_INIT_LEARNED: after a converged step the guess is the net's
 * proposal from G and the previous converged density, floored and
 * renormalised to N_e; before any converged
 * step, or when the proposal is not finite, the plain guess (one-center, or
 * uniform when that rings negative) is used and arche_result.used_fallback is
 * set.  The context does not own the net. */
arche_status arche_set_init_net(arche_ctx *ctx, arche_net *net);

/* The network's guide for the next MD step, without solving: G = n0 + the
 * one-center superposition's change (Sec. 2.5.1's profile from the context's
 * converged step, applied to the structure-factor change from the converged
 * positions to next_pos_host), into guide_host [Nx][Ny][Nz].  Training
 * samples pair it with the previous converged density and the density the next
 * solve converges to.  The converged state, its positions and forces stay as
 * they were; the context's input density (used by ARCHE_INIT_KEEP) is
 * replaced by the plain guess at next_pos_host.  ESTATE without a converged
 * step. */
arche_status arche_learned_guide(arche_ctx *ctx, const double *next_pos_host, double *guide_host);

#ifdef __cplusplus
}
#endif

#endif /* ARCHE_NET_H */
