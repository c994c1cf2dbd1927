/*
 * surrogate.h -- C ABI of the learned surrogate's operations in libsslbm.so:
 * a convolutional network that advances the SEIRD state of the SSLBM
 * (arXiv 2603.19789, Eq. (sslbm_final_clean)) by a fixed number of steps,
 * trained on the GPU on states produced by the SSLBM itself. The paper has
 * no surrogate; these are standard deep-learning operations, on BF16 MFMA
 * with FP32 accumulation.
 *
 * Conventions (as sslbm.h): sslbm_status codes from sslbm.h, host-side
 * validation before any HIP call, caller-owned device buffers, work enqueued
 * on hip_stream (a hipStream_t as void*, NULL = default stream). One
 * difference: where an entry below says that views may not overlap, that is
 * not checked (no SSLBM_E_ALIAS here). Views are often channel slices of
 * one wider buffer, whose byte ranges interleave without sharing an
 * element; overlapping views give undefined results.
 *
 * Tensors
 * -------
 * - Activation views: BF16 (stored as uint16), NHWC. Element (n, y, x, c) of a
 *   view is at p[((n h + y) w + x) pitch + c]. pitch >= channels; channels,
 *   pitch and the view's start (in elements from a 16-byte aligned buffer)
 *   are multiples of 8, and the pointer itself is 16-byte aligned. A view
 *   may be a channel slice of a wider buffer (pitch > channels).
 * - Weights: BF16 [cout][9][cin], tap = 3 (dy + 1) + (dx + 1) for the
 *   neighbour (y + dy, x + dx); bias FP32 [cout].
 * - Convolutions are 3x3 cross-correlations with periodic padding:
 *   y[n,y,x,o] = b[o] + sum_{dy,dx,i} W[o,tap,i] x[n,(y+dy) mod h,(x+dx) mod w,i].
 * - Densities: FP32 [batch][5][h][w] (the SSLBM layout, S E I R D).
 * Errors: SSLBM_E_ARG (NULL pointer, size <= 0, a channel count, pitch or
 * pointer not meeting the alignment above, odd h or w where halving is
 * needed, w not a multiple of 8 for the weight gradient, workspace too
 * small, an input view of a convolution or of its gradients (x, dz)
 * spanning 2 GiB or more: ((n h w - 1) pitch + channels) * 2 >= 2^31
 * bytes), SSLBM_E_HIP.
 */
#ifndef SSLBM_SURROGATE_H
#define SSLBM_SURROGATE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SUR_LEAKY 1   /* apply y = z > 0 ? z : slope z after the bias */
#define SUR_OUT_F32 2 /* write the output view in FP32 instead of BF16 */

/* Forward convolution (see above); y may not overlap x. */
sslbm_status sur_conv3x3_forward(const void *x, int x_pitch, int n, int h, int w, int cin,
                                 const void *weight, const float *bias, void *y, int y_pitch,
                                 int cout, int flags, float slope, void *hip_stream);

/* The forward convolution (BF16 output; SUR_OUT_F32 is rejected) followed
 * by 2 x 2 average pooling of its output: y as sur_conv3x3_forward and
 * `pooled` (n, h/2, w/2; BF16 view of cout channels) as sur_pool2 of y, bit
 * for bit, in one pass where the image allows it. h and w even; neither
 * output may overlap x or each other. */
sslbm_status sur_conv3x3_forward_pool(const void *x, int x_pitch, int n, int h, int w, int cin,
                                      const void *weight, const float *bias, void *y, int y_pitch,
                                      int cout, int flags, float slope, void *pooled,
                                      int pooled_pitch, void *hip_stream);

/* The forward convolution (BF16 output; flags: SUR_LEAKY only) of the
 * channel concatenation [up2(xu), x]: input channels [0, cu) are `xu`
 * (n, h/2, w/2; a BF16 view of cu channels) upsampled 2x by repetition,
 * channels [cu, cin) are `x` (a view of cin - cu channels), without
 * materialising the upsampled tensor. Bit for bit sur_up2 into a
 * concatenation buffer followed by sur_conv3x3_forward. cu a multiple of
 * 32 and less than cin; h, w even. SSLBM_E_UNSUPPORTED for images under
 * 8 x 32 pixels (the caller upsamples explicitly there). */
sslbm_status sur_conv3x3_forward_up(const void *xu, int xu_pitch, int cu, const void *x,
                                    int x_pitch, int n, int h, int w, int cin, const void *weight,
                                    const float *bias, void *y, int y_pitch, int cout, int flags,
                                    float slope, void *hip_stream);

/* dx = d(sum dz * conv(x)) / dx for weight [cout][9][cin]: the convolution
 * of dz with the weights flipped in space and transposed in channels, built
 * in `flip_scratch` (device, >= 18 cout cin bytes). dx is overwritten. */
sslbm_status sur_conv3x3_backward_data(const void *dz, int dz_pitch, int n, int h, int w, int cout,
                                       const void *weight, int cin, void *dx, int dx_pitch,
                                       void *flip_scratch, void *hip_stream);

/* The backward-data weights of several layers in one launch: for each
 * layer l < layers (at most 32), weight[l] ([cout[l]][9][cin[l]], BF16)
 * flipped in space and transposed in channels into flipped[l]
 * ([cin[l]][9][cout[l]], 18 cout cin bytes, 16-byte aligned):
 * flipped[i][8 - tap][o] = weight[o][tap][i]. Host arrays of device
 * pointers; no flipped buffer may overlap a weight or another flipped one.
 * Exact (a permutation). */
sslbm_status sur_flip_weights(int layers, const void *const *weight, const int *cout,
                              const int *cin, void *const *flipped, void *hip_stream);

/* sur_conv3x3_backward_data on weights flipped by sur_flip_weights, and,
 * when act is not NULL, through the adjoint of the leaky activation whose
 * output act is: act is a BF16 view of cin channels at dx's pixels, and
 * each stored value v becomes BF16(act > 0 ? v : slope v). Bit for bit
 * sur_conv3x3_backward_data followed by sur_leaky_backward in place (the
 * chain rule through an activation that feeds this convolution's input,
 * without a separate pass). dx may not overlap dz or act. */
sslbm_status sur_conv3x3_backward_data_flipped(const void *dz, int dz_pitch, int n, int h, int w,
                                               int cout, const void *flipped, int cin, void *dx,
                                               int dx_pitch, const void *act, int act_pitch,
                                               float slope, void *hip_stream);

/* The backward-data pass of a decoder's first convolution, whose first cu
 * input channels were the 2x nearest upsampling of a half-resolution
 * tensor u (the upsampled-input convolution sur_conv3x3_forward_up), in one
 * pass. dx, a view of cin - cu channels, receives the gradient of input
 * channels [cu, cin) (channel c at dx's channel c - cu). du (n, h/2, w/2, cu
 * channels) receives the gradient of u: each 2x2 window of the upsampled
 * channels' BF16-rounded gradient summed, rounded to BF16 and, when du_act
 * is not NULL, passed through the leaky activation's adjoint with du_act (a
 * BF16 view of cu channels at du's pixels, the activation's output). Bit
 * for bit sur_conv3x3_backward_data_flipped into a cin-channel buffer,
 * followed by sur_up2_backward_act (or sur_up2_backward) from its first cu
 * channels into du. cu: a multiple of 16, below cin; h and w even. Images
 * under 8 x 32 pixels return SSLBM_E_UNSUPPORTED (run the two calls above
 * instead). dx and du may not overlap dz, each other or du_act. */
sslbm_status sur_conv3x3_backward_data_up(const void *dz, int dz_pitch, int n, int h, int w,
                                          int cout, const void *flipped, int cin, int cu,
                                          void *dx, int dx_pitch, void *du, int du_pitch,
                                          const void *du_act, int du_act_pitch, float slope,
                                          void *hip_stream);

/* Workspace bytes of sur_conv3x3_backward_weight for these sizes (0 if invalid). */
size_t sur_conv3x3_backward_weight_workspace(int n, int h, int w, int cin, int cout);

/* dweight[o][tap][i] = sum_{n,y,x} dz[n,y,x,o] x[n,y+dy,x+dx,i] and
 * dbias[o] = sum dz[..., o] (FP32, overwritten; dbias may be NULL).
 * Deterministic: FP32 partial sums over pixel ranges added in a fixed order. */
sslbm_status sur_conv3x3_backward_weight(const void *x, int x_pitch, const void *dz, int dz_pitch,
                                         int n, int h, int w, int cin, int cout, float *dweight,
                                         float *dbias, void *workspace, size_t workspace_bytes,
                                         void *hip_stream);

/* sur_conv3x3_backward_weight of the convolution that sur_conv3x3_forward_up
 * computes: its input's channels [0, cu) are xu (n, h/2, w/2) upsampled 2x
 * by repetition and channels [cu, cin) are x, read without the upsampled
 * copy. Bit for bit sur_up2 into a concatenation buffer followed by
 * sur_conv3x3_backward_weight; the same workspace size. cu a multiple of 32
 * and less than cin; h even, w a multiple of 8. SSLBM_E_UNSUPPORTED for
 * images under 8 x 32 pixels. */
sslbm_status sur_conv3x3_backward_weight_up(const void *xu, int xu_pitch, int cu, const void *x,
                                            int x_pitch, const void *dz, int dz_pitch, int n, int h,
                                            int w, int cin, int cout, float *dweight, float *dbias,
                                            void *workspace, size_t workspace_bytes,
                                            void *hip_stream);

/* The weight gradient of sur_conv3x3_backward_weight (xu NULL, cu 0) or of
 * sur_conv3x3_backward_weight_up (xu not NULL), in two stream-ordered parts
 * so that the second overlaps the caller's later work: the per-split
 * partial sums are computed on hip_stream into the workspace; then `event`
 * (a hipEvent_t as void*, created by the caller) is recorded on hip_stream,
 * sum_stream waits for it, and the fixed-order sums over the splits that
 * write dweight and dbias run on sum_stream. The same bits as the one-stream
 * call. dweight, dbias and the workspace belong to the call until the
 * caller has waited for sum_stream; each call in flight needs its own
 * workspace. sum_stream may equal hip_stream (then event may be NULL). */
sslbm_status sur_conv3x3_backward_weight_overlap(const void *xu, int xu_pitch, int cu,
                                                 const void *x, int x_pitch, const void *dz,
                                                 int dz_pitch, int n, int h, int w, int cin,
                                                 int cout, float *dweight, float *dbias,
                                                 void *workspace, size_t workspace_bytes,
                                                 void *hip_stream, void *sum_stream, void *event);

/* dz = y > 0 ? dy : slope dy over `pixels` pixels of c channels (y is the
 * activation's output). dz may alias dy. */
sslbm_status sur_leaky_backward(const void *dy, int dy_pitch, const void *y, int y_pitch, void *dz,
                                int dz_pitch, long long pixels, int c, float slope,
                                void *hip_stream);

/* 2x2 average pooling of x (n, h, w, c) into y (n, h/2, w/2, c), and its
 * adjoint: dx (n, h, w) = dy / 4 broadcast over each window, added to dx
 * when accumulate != 0. */
sslbm_status sur_pool2(const void *x, int x_pitch, int n, int h, int w, int c, void *y, int y_pitch,
                       void *hip_stream);
sslbm_status sur_pool2_backward(const void *dy, int dy_pitch, int n, int h, int w, int c, void *dx,
                                int dx_pitch, int accumulate, void *hip_stream);
/* sur_pool2_backward, then the activation adjoint of sur_leaky_backward on
 * the stored result, with act (a BF16 view of c channels at dx's pixels,
 * not NULL) the activation's output: bit for bit the two calls in a row. */
sslbm_status sur_pool2_backward_act(const void *dy, int dy_pitch, int n, int h, int w, int c,
                                    void *dx, int dx_pitch, int accumulate, const void *act,
                                    int act_pitch, float slope, void *hip_stream);

/* 2x nearest-neighbour upsampling of x (n, h, w, c) into y (n, 2h, 2w, c),
 * and its adjoint: dx (n, h, w) = sum of dy over each 2x2 window. */
sslbm_status sur_up2(const void *x, int x_pitch, int n, int h, int w, int c, void *y, int y_pitch,
                     void *hip_stream);
sslbm_status sur_up2_backward(const void *dy, int dy_pitch, int n, int h, int w, int c, void *dx,
                              int dx_pitch, void *hip_stream);
/* sur_up2_backward, then the activation adjoint as in
 * sur_pool2_backward_act (act a BF16 view of c channels at dx's pixels,
 * not NULL): bit for bit the two calls in a row. */
sslbm_status sur_up2_backward_act(const void *dy, int dy_pitch, int n, int h, int w, int c,
                                  void *dx, int dx_pitch, const void *act, int act_pitch,
                                  float slope, void *hip_stream);

/* Network input from densities: x (BF16 NHWC, 16 channels, pitch 16) holds
 * rho_c / scale_in[c] for c < 5, then planes[b][0..8] (FP32 device
 * [batch][9], the normalised rates and diffusivities) on every pixel, then
 * two zero channels. scale_in: host array of 5 positive floats. */
sslbm_status sur_pack_input(const float *rho, int batch, int h, int w, const float *planes,
                            const float *scale_in, void *x, void *hip_stream);

/* rho_next = rho + scale_out[c] * out[..., c] for c < 5; out is FP32 NHWC
 * with 16 channels (the network's last layer). rho_next may alias rho. */
sslbm_status sur_apply_output(const float *rho, const float *out, int batch, int h, int w,
                              const float *scale_out, float *rho_next, void *hip_stream);

/* Training loss: the mean over (b, y, x, c < 5) of
 * (out[..., c] - (target - rho)_c / scale_out[c])^2 into *loss (device
 * double), and its gradient dout (BF16 NHWC, 16 channels, zero for c >= 5).
 * partials: device scratch of 1024 doubles. */
sslbm_status sur_mse_loss(const float *out, const float *rho, const float *target, int batch, int h,
                          int w, const float *scale_out, void *dout, double *partials, double *loss,
                          void *hip_stream);

/* One Adam step (Kingma and Ba, 2015) over count FP32 parameters; step
 * counts from 1. theta_bf16 (may be NULL) receives the rounded parameters. */
sslbm_status sur_adam(float *theta, void *theta_bf16, const float *grad, float *m, float *v,
                      long long count, int step, float lr, float beta1, float beta2, float eps,
                      void *hip_stream);

/* Periodic crop of a density state: dst[c][j][i] = rho[c][(y0 + j) mod h]
 * [(x0 + i) mod w] for the 5 compartments, j < ch, i < cw (FP32; any integer
 * y0, x0). Used to recompute SSLBM steps on sub-tiles when judging the
 * surrogate. */
sslbm_status sur_crop_periodic(const float *rho, int h, int w, int y0, int x0, int ch, int cw,
                               float *dst, void *hip_stream);

/* dst = round-to-nearest-even BF16 of src (count values). */
sslbm_status sur_to_bf16(const float *src, void *dst, long long count, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SSLBM_SURROGATE_H */
