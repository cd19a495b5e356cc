/*
 * clb_nn.h - C ABI of the learned warm start: the kernels of a convolutional
 * encoder-decoder that predicts a cavity's steady (u, v, T) fields from its
 * porosity map and dimensionless groups, and of its training (mean-squared
 * error, AdamW).  The prediction initialises the lattice Boltzmann solver
 * through clb_set_state_device (clb.h), i.e. f = f^eq(1, u) (Eq. 19) and
 * g = g^eq(T, u) (Eq. 34).  The paper itself starts every run from rest; the
 * network is an addition for many-query use and does not change the steady
 * state the solver converges to.
 *
 * Conventions (all entry points):
 *   - Every pointer is device memory owned by the caller; no call allocates.
 *     `stream` is a hipStream_t passed as void* (NULL: the null stream); all
 *     calls only enqueue work and return without synchronizing.
 *   - Activations are NHWC (batch, height, width, channels; channels
 *     fastest) bfloat16 (clb_bf16 holds the bit pattern); channel counts are
 *     multiples of 16 and tensor base addresses 16-byte aligned.
 *   - Arithmetic: bfloat16 inputs, matrix-core (MFMA) products, FP32
 *     accumulation; stored bfloat16 values are rounded to nearest even.
 *   - Returns CLB_OK, CLB_ERR_ARG for invalid sizes, pointers or alignment
 *     (nothing enqueued), or CLB_ERR_HIP when a launch fails.
 */
#ifndef CLB_NN_H
#define CLB_NN_H

#include <stddef.h>
#include <stdint.h>

#include "clb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef uint16_t clb_bf16;

/* Most layers of the one-launch calls below. */
#define CLB_NN_MAX_LAYERS 64

/* 3x3 convolution, stride 1, zero padding 1:
 *   y[b,i,j,o] = act(bias[o] + sum_{t,c} w[o,t,c] x[b, i+di_t, j+dj_t, c]),
 * taps t = 3 (di + 1) + (dj + 1).  x: (batch, h, w, cin); weight:
 * (cout, 9, cin) bfloat16; bias: cout FP32 values or NULL; act 0 = none,
 * 1 = leaky ReLU with the given slope.  y: (batch, h, w, cout), FP32 when
 * y_fp32 != 0, else bfloat16.  The gradient with respect to the input is
 * this same call on dy with the weights of clb_nn_weights_bf16's w_bwd,
 * no bias and no activation. */
clb_status clb_nn_conv3x3(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w, int32_t cin,
                          const clb_bf16 *weight, const float *bias, int32_t cout, int32_t act,
                          float slope, void *y, int32_t y_fp32, void *stream);

/* The convolution of clb_nn_conv3x3 on the channel concatenation of a
 * decoder level, cin = ca + cb: input channels [0, ca) are tensor a,
 * nearest-neighbour upsampled by 2 when up_a != 0 (a is (batch, h/2, w/2,
 * ca); h and w even), else a as it is ((batch, h, w, ca)); channels
 * [ca, cin) are tensor b, (batch, h, w, cb).  The upsampled and the
 * concatenated tensors are never formed: the operand gather reads a and b.
 * ca and cb multiples of 16, a and b 16-byte aligned; weight (cout, 9, cin).
 * Results are bit-identical to clb_nn_conv3x3 on the formed concatenation. */
clb_status clb_nn_conv3x3_cat(const clb_bf16 *a, int32_t ca, int32_t up_a, const clb_bf16 *b,
                              int32_t cb, int32_t batch, int32_t h, int32_t w,
                              const clb_bf16 *weight, const float *bias, int32_t cout,
                              int32_t act, float slope, void *y, int32_t y_fp32, void *stream);

/* clb_nn_conv3x3 without bias or activation, bfloat16 output split by
 * channels: output channels [0, split) go to y0 (batch, h, w, split), the
 * others to y1 (batch, h, w, cout - split); split a multiple of 16 in
 * (0, cout).  With the w_bwd weights of a concatenated input's convolution
 * it writes the input gradients of the two parts directly. */
clb_status clb_nn_conv3x3_split(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w,
                                int32_t cin, const clb_bf16 *weight, int32_t cout, int32_t split,
                                clb_bf16 *y0, clb_bf16 *y1, void *stream);

/* Gradients of sum(dy * conv3x3(x)) with respect to the weights and bias:
 *   dweight[o,t,c] = sum_{b,i,j} dy[b,i,j,o] x[b, i+di_t, j+dj_t, c],
 *   dbias[o]       = sum_{b,i,j} dy[b,i,j,o]   (dbias may be NULL),
 * both FP32, overwritten.  The sum over pixels is split into chunks whose
 * partial sums go to `workspace` (clb_nn_wgrad_workspace_bytes) and are then
 * added in a fixed order: results are bit-reproducible.  dy and x must be
 * 16-byte aligned; cin and cout multiples of 16 (else CLB_ERR_ARG). */
clb_status clb_nn_wgrad_workspace_bytes(int32_t batch, int32_t h, int32_t w, int32_t cin,
                                        int32_t cout, size_t *bytes);
clb_status clb_nn_conv3x3_wgrad(const clb_bf16 *dy, const clb_bf16 *x, int32_t batch, int32_t h,
                                int32_t w, int32_t cin, int32_t cout, float *dweight,
                                float *dbias, void *workspace, size_t bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the weight
 * gradient of clb_nn_conv3x3_wgrad without a workspace argument.  The partial
 * sums go to a scratch array of clb_nn_wgrad_static_max_bytes() bytes
 * (32 MiB) that the library holds in each GPU's memory from its first use on
 * that GPU until the process ends; the call allocates nothing.  Sizes whose
 * clb_nn_wgrad_workspace_bytes exceeds that maximum return CLB_ERR_WORKSPACE
 * (nothing enqueued); every layer of the 5-level network at batch 32 on
 * 128 x 128 images fits (18 MiB at most).  All calls on one GPU share its
 * scratch array: calls that overlap in time on one GPU (different streams,
 * or host threads) race and must be serialized by the caller.  Results are
 * bit-identical to clb_nn_conv3x3_wgrad's.  Other arguments and errors as
 * clb_nn_conv3x3_wgrad. */
size_t clb_nn_wgrad_static_max_bytes(void);
clb_status clb_nn_conv3x3_wgrad_static(const clb_bf16 *dy, const clb_bf16 *x, int32_t batch,
                                       int32_t h, int32_t w, int32_t cin, int32_t cout,
                                       float *dweight, float *dbias, void *stream);

/* clb_nn_conv3x3_wgrad for the concatenated input of clb_nn_conv3x3_cat
 * (same a, ca, up_a, b, cb; workspace of clb_nn_wgrad_workspace_bytes with
 * cin = ca + cb).  Bit-identical to clb_nn_conv3x3_wgrad on the formed
 * concatenation. */
clb_status clb_nn_conv3x3_wgrad_cat(const clb_bf16 *dy, const clb_bf16 *a, int32_t ca,
                                    int32_t up_a, const clb_bf16 *b, int32_t cb, int32_t batch,
                                    int32_t h, int32_t w, int32_t cout, float *dweight,
                                    float *dbias, void *workspace, size_t bytes, void *stream);

/* The weight gradient in two steps, so that the chunk sums of many layers
 * are added in one launch: clb_nn_conv3x3_wgrad_parts (and _cat_parts, the
 * arguments of clb_nn_conv3x3_wgrad and clb_nn_conv3x3_wgrad_cat) only leave
 * the per-chunk partial sums in `workspace` (16-byte aligned, at least
 * clb_nn_wgrad_workspace_bytes), the bias sums too when with_bias != 0, and
 * store their chunk count in *nsplit (a host int32).  The workspace must stay
 * untouched until clb_nn_wgrad_reduce_layers has read it: for layer l it
 * adds the nsplit[l] chunks at parts[l] (a layer of cout[l] outputs and
 * cin[l] inputs) into dweight[l] and, when dbias[l] is not NULL (allowed
 * only for partials taken with with_bias), dbias[l].  parts, nsplit, cout,
 * cin, dweight and dbias are host arrays of nlayers entries (1 <= nlayers <=
 * CLB_NN_MAX_LAYERS) holding device pointers.  The sums are bit-identical to
 * those of clb_nn_conv3x3_wgrad. */
clb_status clb_nn_conv3x3_wgrad_parts(const clb_bf16 *dy, const clb_bf16 *x, int32_t batch,
                                      int32_t h, int32_t w, int32_t cin, int32_t cout,
                                      int32_t with_bias, void *workspace, size_t bytes,
                                      int32_t *nsplit, void *stream);
clb_status clb_nn_conv3x3_wgrad_cat_parts(const clb_bf16 *dy, const clb_bf16 *a, int32_t ca,
                                          int32_t up_a, const clb_bf16 *b, int32_t cb,
                                          int32_t batch, int32_t h, int32_t w, int32_t cout,
                                          int32_t with_bias, void *workspace, size_t bytes,
                                          int32_t *nsplit, void *stream);
clb_status clb_nn_wgrad_reduce_layers(int32_t nlayers, void *const *parts, const int32_t *nsplit,
                                      const int32_t *cout, const int32_t *cin,
                                      float *const *dweight, float *const *dbias, void *stream);

/* bfloat16 copies of FP32 master weights (cout, 9, cin): w_fwd in the same
 * layout, w_bwd = the weights of the input-gradient convolution, laid out
 * (cin, 9, cout) with the taps reversed: w_bwd[c, 8 - t, o] = w[o, t, c]. */
clb_status clb_nn_weights_bf16(const float *w32, int32_t cout, int32_t cin, clb_bf16 *w_fwd,
                               clb_bf16 *w_bwd, void *stream);

/* clb_nn_weights_bf16 for the nlayers convolutions of one flat parameter
 * array, in one launch: layer l has cout[l] x 9 x cin[l] weights starting at
 * element offset[l] of w32, and its two bfloat16 copies start at the same
 * element offset of w_fwd and w_bwd (arrays as long as w32; elements outside
 * the layers' weights are left unchanged).  cout, cin and offset are host
 * arrays of nlayers entries, 1 <= nlayers <= CLB_NN_MAX_LAYERS; the layers
 * must not overlap. */
clb_status clb_nn_weights_bf16_layers(const float *w32, int32_t nlayers, const int32_t *cout,
                                      const int32_t *cin, const int64_t *offset,
                                      clb_bf16 *w_fwd, clb_bf16 *w_bwd, void *stream);

/* 2x2 average pooling of x (batch, h, w, c) into (batch, h/2, w/2, c), h and w
 * even; and its gradient dx[b,i,j,c] = dy[b,i/2,j/2,c] / 4. */
clb_status clb_nn_pool2(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w, int32_t c,
                        clb_bf16 *y, void *stream);
clb_status clb_nn_pool2_grad(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w, int32_t c,
                             clb_bf16 *dx, void *stream);

/* Nearest-neighbour 2x upsampling of x (batch, h, w, c) into (batch, 2h, 2w,
 * c); and its gradient dx[b,i,j,c] = sum of dy over the 2x2 block. */
clb_status clb_nn_up2(const clb_bf16 *x, int32_t batch, int32_t h, int32_t w, int32_t c,
                      clb_bf16 *y, void *stream);
clb_status clb_nn_up2_grad(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w, int32_t c,
                           clb_bf16 *dx, void *stream);

/* Channel concatenation y[p] = [a[p] (ca channels), b[p] (cb channels)] over
 * npix pixels, and its inverse split. */
clb_status clb_nn_concat(const clb_bf16 *a, int32_t ca, const clb_bf16 *b, int32_t cb,
                         int64_t npix, clb_bf16 *y, void *stream);
clb_status clb_nn_split(const clb_bf16 *y, int32_t ca, int32_t cb, int64_t npix, clb_bf16 *a,
                        clb_bf16 *b, void *stream);

/* Gradient through a leaky ReLU output `out` that feeds one or two consumers:
 *   s = g0 + g1 (g1 may be NULL), rounded to bfloat16;
 *   dz = s (out > 0) or slope * s (otherwise), rounded to bfloat16. */
clb_status clb_nn_act_grad(const clb_bf16 *g0, const clb_bf16 *g1, const clb_bf16 *out,
                           int64_t n, float slope, clb_bf16 *dz, void *stream);

/* The input gradient of a convolution, the pooling gradient and the
 * upsampling gradient, each followed by the gradient through the leaky ReLU
 * whose output y (bfloat16) has the result's layout, for a tensor whose
 * gradient is complete with this contribution:
 *   clb_nn_conv3x3_act_grad: r = clb_nn_conv3x3(dy, ..., weight, no bias, no
 *     activation) rounded to bfloat16;
 *   clb_nn_pool2_grad_act: r = clb_nn_pool2_grad(dy), plus the tensor's
 *     other contribution `add` (may be NULL) as clb_nn_act_grad adds it;
 *   clb_nn_up2_grad_act: r = clb_nn_up2_grad(dy);
 * then dz = r (y > 0) or slope * r, rounded to bfloat16: bit-identical to the
 * unfused call followed by clb_nn_act_grad.  The pooling and upsampling
 * variants need c a multiple of 8 and 16-byte aligned tensors. */
clb_status clb_nn_conv3x3_act_grad(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w,
                                   int32_t cin, const clb_bf16 *weight, int32_t cout,
                                   const clb_bf16 *y, float slope, clb_bf16 *dz, void *stream);
clb_status clb_nn_pool2_grad_act(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w,
                                 int32_t c, const clb_bf16 *add, const clb_bf16 *y, float slope,
                                 clb_bf16 *dz, void *stream);
clb_status clb_nn_up2_grad_act(const clb_bf16 *dy, int32_t batch, int32_t h, int32_t w, int32_t c,
                               const clb_bf16 *y, float slope, clb_bf16 *dz, void *stream);

/* Mean-squared error over the first nch channels of an FP32 output with row
 * stride ldo (channels per pixel) against targets (npix, nch) FP32:
 *   loss = mean((out - target)^2) (FP64, written to *d_loss on the device),
 *   dout[p, c] = 2 (out - target) / (npix nch) for c < nch, 0 for other c,
 * bfloat16 with row stride ldo.  ldo is a multiple of 8 and out, dout are
 * 16-byte aligned.  workspace: clb_nn_mse_workspace_bytes. */
clb_status clb_nn_mse_workspace_bytes(int64_t npix, size_t *bytes);
clb_status clb_nn_mse(const float *out, int32_t ldo, const float *target, int32_t nch,
                      int64_t npix, clb_bf16 *dout, double *d_loss, void *workspace,
                      size_t bytes, void *stream);

/* AdamW step t >= 1 on n FP32 parameters (decoupled weight decay, bias-
 * corrected moments; Loshchilov & Hutter):
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   p -= lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd p). */
clb_status clb_nn_adamw(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                        float b1, float b2, float eps, float wd, int32_t t, void *stream);

/* clb_nn_adamw followed, in the same launch, by the bfloat16 copies of
 * clb_nn_weights_bf16_layers for the updated parameters (same layer table;
 * the offsets must increase and every layer lie within the n parameters). */
clb_status clb_nn_adamw_layers(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                               float b1, float b2, float eps, float wd, int32_t t,
                               int32_t nlayers, const int32_t *cout, const int32_t *cin,
                               const int64_t *offset, clb_bf16 *w_fwd, clb_bf16 *w_bwd,
                               void *stream);

/* Network input for `batch` samples picked by idx (device int32, indices into
 * the sample arrays): channel 0 = (eps - 0.625) * 5 from the porosity maps
 * eps_all (samples, h, w) FP32; channels 1..ngroups = groups_all[s, k]
 * (samples, ngroups) FP32, normalised dimensionless groups, constant over the
 * image; the next two channels = x and y mapped to [-1, 1]; the rest 0.
 * ngroups <= 13.  x: (batch, h, w, 16) bfloat16. */
clb_status clb_nn_features(const float *eps_all, const float *groups_all, int32_t ngroups,
                           const int32_t *idx, int32_t batch, int32_t h, int32_t w,
                           clb_bf16 *x, void *stream);

/* Training targets for the same picks: out[b, p, c] = fields_all[idx[b], p, c]
 * for p < h w, c < nch (FP32). */
clb_status clb_nn_gather(const float *fields_all, int32_t nch, const int32_t *idx,
                         int32_t batch, int64_t npix, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CLB_NN_H */
