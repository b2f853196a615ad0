/*
 * pam_nn.h - C-ABI of the HIP kernels of the NCC-mask surrogate (gfx950).
 *
 * The surrogate predicts the normalised NCC weighting (the NNCC of Sections II-A
 * and II-C) of a frame from its full-aperture angular-spectrum energy (Eq. 3),
 * so that the image I = rho_n^2 * E of Eq. 11 can be formed from one propagation
 * instead of three.  It is a U-Net: 3x3 convolutions, 2x2 max pooling, nearest
 * 2x upsampling, channel concatenation, a 1x1 head with a mask output and a
 * predicted-error (confidence) output, energy-weighted binary cross-entropy losses
 * for the mask and the error head, and Adam.
 *
 * Conventions
 *   Activations: BF16, NHWC ([batch][h][w][channels], channels fastest) with a
 *   channel stride ld >= channels, so a tensor may be a channel slice of a wider
 *   buffer (concatenation without copies).  Channel counts used by the 3x3
 *   kernels are multiples of 32; w is a multiple of 32.
 *   Master weights: FP32 [9][c_in][c_out], tap t = 3 (dh + 1) + (dw + 1); the
 *   convolution is a cross-correlation with zero padding.  Matrix-core products
 *   take BF16 operands and accumulate in FP32.
 *   All pointers are device memory owned by the caller; every call enqueues on
 *   hip_stream (NULL = default stream) and returns PAM_ERR_INVALID_ARG before
 *   enqueuing anything when a size or pointer is invalid.
 */
#ifndef PAM_NN_H
#define PAM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "pam.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv3x3(x) + bias) (or y += conv3x3(x) when accumulate != 0, no bias/act).
 *   x  [batch][h][w] rows of k_in BF16 channels with stride ldx
 *   wt BF16 [n_out][9][k_in]: wt[o][t][c] = W[t][c][o] (pam_nn_pack_weights)
 *   y  [batch][h][w] rows of n_out BF16 channels with stride ldy
 * flip != 0 uses the tap at (-dh, -dw): with wt = the "wd" layout of
 * pam_nn_pack_weights this computes the gradient with respect to the input. */
pam_status_t pam_nn_conv3x3(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t k_in,
                            const void* wt, const float* bias, void* y, int32_t ldy, int32_t n_out,
                            int32_t relu, int32_t flip, int32_t accumulate, void* hip_stream);

/* dW[t][c][o] += sum_pixels x[p + off(t)][c] * dy[p][o]; db[o] += sum_p dy[p][o] (db nullable).
 * dw (FP32 [9][c_in][c_out]) and db are accumulated with atomics: zero them first.
 * x and dy 16-byte aligned, ldx and lddy multiples of 8 (else PAM_ERR_INVALID_ARG); the
 * products run on the matrix cores (BF16 operands, FP32 sums). */
pam_status_t pam_nn_conv3x3_wgrad(const void* x, int32_t ldx, const void* dy, int32_t lddy, int32_t batch,
                                  int32_t h, int32_t w, int32_t c_in, int32_t c_out, float* dw, float* db,
                                  void* hip_stream);

/* dy[p][c] *= (y[p][c] > 0), in place. */
pam_status_t pam_nn_relu_backward(const void* y, int32_t ldy, void* dy, int32_t lddy, int64_t pixels, int32_t c,
                                  void* hip_stream);

/* 2x2 max pooling of x ([batch][h][w], h and w even) into y ([batch][h/2][w/2]);
 * arg (uint8 [batch][h/2][w/2][c]) records the first maximum in the order
 * (0,0), (0,1), (1,0), (1,1). */
pam_status_t pam_nn_maxpool(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t c, void* y,
                            int32_t ldy, uint8_t* arg, void* hip_stream);

/* dx (+)= unpool(dy): each dy value goes to its recorded maximum, zeros elsewhere
 * (accumulate != 0 adds into dx instead of overwriting).  h, w are the sizes of dx. */
pam_status_t pam_nn_maxpool_backward(const void* dy, int32_t lddy, const uint8_t* arg, int32_t batch, int32_t h,
                                     int32_t w, int32_t c, void* dx, int32_t lddx, int32_t accumulate,
                                     void* hip_stream);

/* y[b][h][w] = x[b][h/2][w/2] (nearest 2x); h, w are the sizes of x. */
pam_status_t pam_nn_upsample(const void* x, int32_t ldx, int32_t batch, int32_t h, int32_t w, int32_t c, void* y,
                             int32_t ldy, void* hip_stream);

/* dx[b][h][w] = sum of the 2x2 block of dy; h, w are the sizes of dx. */
pam_status_t pam_nn_upsample_backward(const void* dy, int32_t lddy, int32_t batch, int32_t h, int32_t w, int32_t c,
                                      void* dx, int32_t lddx, void* hip_stream);

/* Head: z_o = b[o] + sum_c feat[p][c] w[c][o] (w FP32 [c][2]); mask = sigmoid(z_0),
 * err = sigmoid(z_1).  With target t (FP32 [pixels]) also the weighted losses
 * (zero loss[0..2] first):
 *   loss[0] += sum_p w_p BCE(mask, t), loss[1] += sum_p w_p BCE(err, |mask - t|),
 *   loss[2] += sum_p w_p |mask - t|   (reported, not differentiated),
 * BCE(s, y) = -y log s - (1 - y) log(1 - s), and the gradient of loss[0] + loss[1]
 * dz (FP32 [pixels][2]) = ((mask - t) w_p, (err - |mask - t|) w_p) with the error
 * target held constant; w_p = weight[p] (FP32 [pixels]) or 1/count when weight
 * is NULL.  target, weight, dz and loss may be NULL (inference). */
pam_status_t pam_nn_head(const void* feat, int32_t c, int64_t pixels, const float* w, const float* b,
                         const float* target, const float* weight, float* mask, float* err, float* dz, float* loss,
                         int64_t count, void* hip_stream);

/* Loss weights w[f][p] = ((1 - mix) E[f][p] / sum_p E[f][p] + mix / pixels) / batch:
 * the loss concentrates where the image I = rho_n^2 E has energy. */
pam_status_t pam_nn_loss_weights(const float* energy, int32_t batch, int64_t pixels, float mix, float* out,
                                 void* hip_stream);

/* Head gradients: dfeat (BF16 [pixels][c]) = dz w^T; dw (FP32 [c][2]) += feat^T dz;
 * db (FP32 [2]) += column sums of dz (zero dw, db first). */
pam_status_t pam_nn_head_backward(const void* feat, int32_t c, int64_t pixels, const float* w, const float* dz,
                                  void* dfeat, float* dw, float* db, void* hip_stream);

/* Adam on FP32 master parameters: m, v moments; step >= 1 (bias correction). */
pam_status_t pam_nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* hip_stream);

/* BF16 layouts of W (FP32 [9][c_in][c_out]): wt[o][t][c] = W[t][c][o] (forward) and
 * wd[c][t][o] = W[t][c][o] (input gradient, used with flip).  wd may be NULL. */
pam_status_t pam_nn_pack_weights(const float* w, int32_t c_in, int32_t c_out, void* wt, void* wd, void* hip_stream);

/* Network input from full-aperture energies E (FP32 [batch][pixels]): BF16
 * [batch][pixels][32] with channel 0 = clamp(log10(E / max E) / 6 + 1, 0, 1),
 * channel 1 = E / max E, channels 2..31 = 0 (max over each frame). */
pam_status_t pam_nn_features(const float* energy, int32_t batch, int64_t pixels, void* out, void* hip_stream);

/* Network input from the accumulator channels of a full-aperture plan built with
 * coherence = 1 (pam.h): accum FP32 [n_split][batch][5][n_z][n_x] (S, Re G_x, Im G_x,
 * Re G_z, Im G_z), consecutive splits split_stride floats apart (ignored when n_split = 1).
 * Writes energy FP32 [batch][n_z][n_x] = S summed over the splits, frame_max FP32 [batch]
 * = its maximum over each frame (caller-owned, overwritten) and BF16
 * [batch][n_z * n_x][32] features:
 *   0: clamp(log10(S / max S) / 6 + 1, 0, 1)        1: S / max S
 *   2-4: |c_x|, Re c_x, Im c_x with c_x = G_x / sqrt(S(z, x0) S(z, x0 + 1)) of the
 *        column pair (x0, x0 + 1), x0 = x rounded down to even
 *   5-7: the same for the depth pair (z0, z0 + 1), z0 = z rounded down to even
 *   8-31: 0
 * A pair whose energies multiply to 0 has c = 0.  n_z and n_x must be even. */
pam_status_t pam_nn_coherence_features(const float* accum, int32_t n_split, int64_t split_stride, int32_t batch,
                                       int32_t n_z, int32_t n_x, void* out, float* energy, float* frame_max,
                                       void* hip_stream);

/* Predicted relative L2 error of each frame's image mask^2 E when the mask is off by
 * err per pixel: est[f] = ||2 mask err E|| / ||mask^2 E|| over the frame's pixels (FP64
 * sums; +inf for an all-zero image).  mask, err, energy FP32 [batch][pixels]. */
pam_status_t pam_nn_error_estimate(const float* mask, const float* err, const float* energy, int32_t batch,
                                   int64_t pixels, float* est, void* hip_stream);

/* Per-frame confidence conf[f] = 1 - sum_p E err / sum_p E (energy-weighted mean of
 * the predicted mask error); err, energy FP32 [batch][pixels]. */
pam_status_t pam_nn_confidence(const float* err, const float* energy, int32_t batch, int64_t pixels, float* conf,
                               void* hip_stream);

/* image[i] = mask[i]^2 * energy[i] (Eq. 11 with the predicted NNCC). */
pam_status_t pam_nn_apply_mask(const float* mask, const float* energy, float* image, int64_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PAM_NN_H */
