/*
 * lbtp_nn.h -- learned warm start of the pressure iteration (MI355X, bf16
 * matrix cores).  Not part of the paper's method: the network only supplies
 * the initial pressure P0 handed to lbtp_set_state / lbtp_batch_set_state;
 * the lattice Boltzmann pressure iteration (eq. 3-1) then runs to the same
 * stopping tolerance as from any other start, so it still decides the result.
 *
 * Network: convolutional encoder-decoder on an N x H x W batch of fields.
 * Inputs per node: lnK (log absolute permeability), S (saturation) and the
 * proximity exp(-d/16) of the nearer Dirichlet wall (d = min(x + 1/2,
 * W - x - 1/2) nodes; flow axis x, pressure 1 at x = 0 and 0 at x = W).
 * Output: P = (1 - (x + 1/2)/W) + (scale / W) * net, so the learned part is
 * per node and a network trained on one grid size applies to others.  `levels` resolution
 * levels with base * 2^l channels, two 3x3 convolutions + ReLU per level and
 * side, 2x2 average pooling, nearest 2x upsampling, concatenated skips, 3x3
 * head.  Parameters: one flat float32 vector, per convolution the weights
 * [Co][3][3][Ci] then the bias [Co], convolutions in forward order (encoder
 * levels 0..levels-1, decoder levels levels-2..0, head).  Activations are
 * bf16, products accumulate in float32 (MFMA), master weights, gradients and
 * Adam moments are float32.
 *
 * Fields are float32 arrays [N][H][W] (x fastest).  H and W must be
 * multiples of 2^(levels-1).  on_device as in lbtp.h.  Calls run on the
 * stream given at creation and return after it has finished.  Errors:
 * LBTP_EINVAL (bad argument or shape), LBTP_ENOMEM, LBTP_EHIP.
 */
#ifndef LBTP_NN_H
#define LBTP_NN_H

#include "lbtp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbtp_nn lbtp_nn;

/* New network with all parameters zero (set them with lbtp_nn_set_params). */
LBTP_API int lbtp_nn_create(int base, int levels, double scale, void *stream, lbtp_nn **out);
LBTP_API void lbtp_nn_destroy(lbtp_nn *nn);
LBTP_API long long lbtp_nn_num_params(lbtp_nn *nn);
/* Replace / read the flat parameter vector; set_params also resets Adam. */
LBTP_API int lbtp_nn_set_params(lbtp_nn *nn, const float *theta, int on_device);
LBTP_API int lbtp_nn_get_params(lbtp_nn *nn, float *theta, int on_device);
/* P [N][H][W] from lnK and S.  With factor > 1 the network runs on the grid
 * coarsened by `factor` (lnK and S averaged over factor x factor blocks, so
 * the coarse permeability is the geometric block mean); the coarse deviation
 * from the linear profile is interpolated bilinearly to the fine node centres
 * (coarse coordinate (x + 1/2)/factor - 1/2, clamped at the edges) and added
 * to the fine linear profile.  This gives a network trained on one grid size
 * the long-wavelength pressure modes of a larger grid, which are the slowest
 * to converge.  h and w must be multiples of factor, and h/factor and
 * w/factor multiples of 2^(levels-1). */
LBTP_API int lbtp_nn_predict(lbtp_nn *nn, const float *lnK, const float *S, int n, int h, int w, int factor,
                             float *P, int on_device);
/* lbtp_nn_predict without any device allocation, for callers that cannot
 * allocate: code being captured into a HIP graph, tight serving loops, hosts
 * that forbid hipMalloc.  Same result as lbtp_nn_predict (the same kernels
 * in the same order).  lnK, S and P are device pointers of the current
 * device; the activations, the head output and the coarsened inputs live in
 * a static device array of LBTP_NN_SCRATCH_BYTES per device, held from
 * library load until the process ends (its address is looked up once per
 * device, at lbtp_nn_create or at the first call on another device).  A
 * shape whose buffers do not fit -- about 1.2 kB per coarse node
 * n * (h/factor) * (w/factor) with base 32 and 4 levels, so up to 128 x 128
 * coarse nodes -- is rejected with LBTP_EINVAL before anything is launched.
 * Every call on one device shares that array: calls that overlap on one
 * device (several streams, several threads) race and must be serialised by
 * the caller.  Enqueued on the network's stream; does not synchronise. */
#define LBTP_NN_SCRATCH_BYTES (32ll << 20)
LBTP_API int lbtp_nn_predict_noalloc(lbtp_nn *nn, const float *lnK, const float *S, int n, int h, int w, int factor,
                                     float *P);
/* Weighted mean squared error L = (1 / (n h w)) sum_k weight[k] sum_nodes
 * (P_net - P)^2 against the target P, and its gradient (flat, may be NULL).
 * weight: one float per sample, or NULL for all ones. */
LBTP_API int lbtp_nn_loss_grad(lbtp_nn *nn, const float *lnK, const float *S, const float *P, const float *weight,
                               int n, int h, int w, double *loss, float *grad, int on_device);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss; *loss (may
 * be NULL) receives the loss before the step. */
LBTP_API int lbtp_nn_train_step(lbtp_nn *nn, const float *lnK, const float *S, const float *P, const float *weight,
                                int n, int h, int w, double lr, double *loss, int on_device);

#ifdef __cplusplus
}
#endif
#endif /* LBTP_NN_H */
