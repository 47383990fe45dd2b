/*
 * polrad_denoiser.h -- C ABI of the learned Stokes-map denoiser in
 * libpolrad.so.
 *
 * The denoiser is not part of the radiative-transfer method of Yang & Wang
 * (arXiv:2512.01283).  It post-processes the Stokes images of two-step
 * imaging (Sec. 2.3): from a map made with few packets it estimates the Q and
 * U of a map made with many more.  Monte Carlo noise falls only as N^-1/2, so
 * a good estimate saves packets.
 *
 * Per image, with s = mean of I over the image and Ihat = I / s, the input
 * features are x = (ln max(Ihat, 1e-6), Q/I, U/I, V/I) (the ratios clamped to
 * [-1, 1], the range of a physical Stokes vector, and 0 where I <= 0).
 * Network: a U-Net of L levels (2..6) with widths c1..cL; every 3x3
 * convolution has zero padding 1, a bias and a relu; a block is two of them.
 * For L = 3:
 *   e1    = block(x, 4->c1)                                  H x W
 *   e2    = block(pool(e1), c1->c2)                          H/2
 *   m3    = block(pool(e2), c2->c3)                          H/4
 *   d2    = block([up(m3), e2], c3+c2->c2)                   H/2
 *   d1    = block([up(d2), e1], c2+c1->c1)                   H
 *   delta = head(d1)        head: 1x1 convolution c1 -> 2
 * and in general encoder blocks e1..e(L-1), each followed by pool, the block
 * mL at H / 2^(L-1), and decoder blocks d(L-1)..d1 on [up(below), e_l].
 * pool = 2x2 mean, up = 2x nearest repeat, [a, b] = channel concatenation
 * (a first).  Predicted fractions q' = Q/I + delta_0, u' = U/I + delta_1;
 * the denoised map is (I, q' I, u' I, V).
 * Training minimises, averaged over the images of a batch, the squared
 * relative Q/U error of the prediction against the target maps (Q_t, U_t):
 *   sum_p [(q' Ihat - Q_t/s)^2 + (u' Ihat - U_t/s)^2] / sum_p Ihat^2
 * (s and Ihat from the input map), by Adam (beta1 0.9, beta2 0.999, eps
 * 1e-8, bias-corrected) on FP32 master weights.
 *
 * Parameters are one flat FP32 array: for each convolution in the order
 * e1a e1b ... e(L-1)a e(L-1)b mLa mLb d(L-1)a d(L-1)b ... d1a d1b
 * (L = 3: e1a e1b e2a e2b m3a m3b d2a d2b d1a d1b) its weights [cout][3][3][cin]
 * (w[o][dy][dx][c] multiplies x[h + dy - 1][w + dx - 1][c]) then its bias
 * [cout]; then the head's weights [2][c1] and bias [2].
 *
 * Arithmetic: convolutions run on BF16 matrix cores with FP32 accumulation
 * (weights and activations rounded to BF16, nearest even); the head, loss,
 * gradients of the weights, the optimiser and the maps are FP32/FP64.
 *
 * Maps are FP64 device arrays [batch][4][height][width] (I, Q, U, V), the
 * layout of kp_get_images_device for one wavelength's views, so images of a
 * run can be passed straight in.
 *
 * Two-run inputs (kp_dn_create_runs with runs = 2): an input image is two
 * independent runs A and B of the same scene with the same packet count,
 * [batch][8][height][width] (A's I, Q, U, V, then B's).  (I, Q, U, V) above
 * are then the two runs' mean -- the map of one run with both runs' packets
 * -- and four more features follow, |S_A - S_B| / (2 I) for S = I, Q, U, V
 * (clamped to [0, 1], 0 where I <= 0): a per-pixel sample of the mean's
 * Monte Carlo noise, which one map alone does not carry.  The first
 * convolution then has cin = 8; the output (kp_dn_infer) and the training
 * targets (kp_dn_backward) stay [batch][4][height][width].  height and width must be multiples of
 * 2^(L-1) (L-1 pooling levels); batch * height * width <= 2^24.
 *
 * Errors follow polrad.h: every call returns kp_status, arguments are
 * validated before any launch, kp_dn_last_error() gives the message.  A
 * handle is bound to one device and is not thread-safe.  Device memory for
 * activations is allocated on first use for a given size and kept.
 */
#ifndef POLRAD_DENOISER_H
#define POLRAD_DENOISER_H
#include <stddef.h>
#include <stdint.h>

#include "polrad.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kp_dn kp_dn;

/* Create a denoiser of the Sec. 2.3 images (not in the paper: the learned
 * part above) of n_levels (2..6) levels with widths[n_levels] (host;
 * each a multiple of 16 in [16, 512]) on HIP device `device`, with all
 * parameters zero.  *out receives an owned handle (release with
 * kp_dn_destroy). */
kp_status kp_dn_create(int device, const int32_t *widths, int32_t n_levels, kp_dn **out);
/* As kp_dn_create for inputs of `runs` (1 or 2) independent runs per image
 * (see two-run inputs above; two Sec. 2.3 imaging runs with independent
 * packet streams); kp_dn_create is runs = 1. */
kp_status kp_dn_create_runs(int device, const int32_t *widths, int32_t n_levels, int32_t runs, kp_dn **out);
/* Release a denoiser handle and its device memory (not in the paper; NULL
 * is ignored), and the message of its last failed call. */
void kp_dn_destroy(kp_dn *dn);
const char *kp_dn_last_error(const kp_dn *dn);

/* Number of FP32 parameters (the length of the flat array above; the
 * learned part, not in the paper). */
kp_status kp_dn_num_params(const kp_dn *dn, size_t *n);
/* Copy n = kp_dn_num_params parameters from / to host memory (learned part,
 * not in the paper).  Setting the parameters clears the Adam moments and step
 * count; KP_ERR_ARG for a wrong n or a non-finite value. */
kp_status kp_dn_set_params(kp_dn *dn, const float *host_params, size_t n);
kp_status kp_dn_get_params(kp_dn *dn, float *host_params, size_t n);
/* Gradient of the loss of the last kp_dn_backward / kp_dn_train_step with
 * respect to every parameter, same layout (host copy of n floats; learned
 * part, not in the paper). */
kp_status kp_dn_get_grads(kp_dn *dn, float *host_grads, size_t n);
/* Adam state for checkpoint and resume (learned part, not in the paper):
 * first and second moments (n floats each, host) and the number of steps
 * taken. */
kp_status kp_dn_get_adam(kp_dn *dn, float *host_m, float *host_v, size_t n, int32_t *step);
kp_status kp_dn_set_adam(kp_dn *dn, const float *host_m, const float *host_v, size_t n, int32_t step);

/* Denoise Sec. 2.3 Stokes images (not in the paper): d_maps (device, read;
 * [batch][4 runs][height][width]) -> d_out (device, written,
 * [batch][4][height][width]; may not alias d_maps).  Asynchronous on
 * hip_stream. */
kp_status kp_dn_infer(kp_dn *dn, const double *d_maps, double *d_out, int32_t batch, int32_t height,
                      int32_t width, void *hip_stream);
/* Test-time averaging (not in the paper; Sec. 2.3 images): as kp_dn_infer,
 * with q' and u' the mean over the eight dihedral transforms of each input
 * (the aug codes of kp_dn_backward) of the network's prediction for the transformed image, mapped back to the
 * original pixels and Stokes signs; only the four codes without a quarter
 * turn when height != width.  Eight (four) forward passes.  The average is
 * exactly equivariant under the group, and by convexity its squared Q/U
 * error is at most the mean of the single passes' squared errors. */
kp_status kp_dn_infer_tta(kp_dn *dn, const double *d_maps, double *d_out, int32_t batch, int32_t height,
                          int32_t width, void *hip_stream);

/* Loss and gradients (not in the paper; pairs of Sec. 2.3 images of the
 * same scene at few and many packets) for the pairs (d_low[b], d_high[b])
 * (device maps; d_low [batch][4 runs][height][width], d_high
 * [batch][4][height][width]).
 * host_aug (NULL = identity) holds one code per image, 0..7, of the
 * dihedral transform applied to both maps of a pair before the network:
 * code a = r + 4 f mirrors the width axis when f = 1, then rotates the image
 * by r quarter turns (numpy's rot90 on the (height, width) axes), and maps
 * Stokes as (Q, U, V) -> ((-1)^r Q, (-1)^(r+f) U, (-1)^f V); odd r needs
 * height == width.  *loss (host) receives the loss above; the call
 * synchronises hip_stream. */
kp_status kp_dn_backward(kp_dn *dn, const double *d_low, const double *d_high, int32_t batch,
                         int32_t height, int32_t width, const int32_t *host_aug, double *loss,
                         void *hip_stream);
/* One Adam step with learning rate lr (> 0) from the gradients of the last
 * kp_dn_backward (learned part, not in the paper).  Asynchronous on
 * hip_stream. */
kp_status kp_dn_adam_step(kp_dn *dn, float lr, void *hip_stream);
/* kp_dn_backward followed by kp_dn_adam_step (learned part, not in the
 * paper). */
kp_status kp_dn_train_step(kp_dn *dn, const double *d_low, const double *d_high, int32_t batch,
                           int32_t height, int32_t width, const int32_t *host_aug, float lr,
                           double *loss, void *hip_stream);

/* Device time of the last kp_dn_infer / kp_dn_backward (learned part, not
 * in the paper), in ms, split into
 * the 3x3 convolution kernels (forward and input gradient), the weight
 * gradient kernels, and everything else; HIP events on the call's stream. */
typedef struct {
  double ms_total;
  double ms_conv;
  double ms_wgrad;
  double ms_other;
  double conv_flop; /* algorithmic FLOP of the convolution kernels timed in ms_conv */
  double wgrad_flop;
} kp_dn_timing;
kp_status kp_dn_get_timing(kp_dn *dn, kp_dn_timing *out);

#ifdef __cplusplus
}
#endif
#endif
