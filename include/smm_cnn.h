/*
 * smm_cnn.h -- C ABI of the learned warm start for batched SMM solves.
 *
 * The SMM fixed point (eq. moment:smm_fp) may start from any scalar flux;
 * the paper starts from an unstated guess (Sec. 5).  This library adds a
 * small convolutional network that predicts, per element of a uniform
 * Cartesian mesh, the nodal correction of the converged scalar flux over the
 * diffusion start and the nodal SMM correction source (the part of the
 * right-hand side of eq. ipsmm built from T and beta).  The start is the
 * diffusion start (the moment system with zero correction source) plus the
 * predicted flux correction; the correction-source channels are an auxiliary
 * training target.  A problem whose prediction is not finite keeps the
 * diffusion start.  The converged answer does not depend on the start.
 *
 * Network: a stack of 3x3 convolutions (zero padding, stride 1), ReLU after
 * every layer but the last, NHWC activations in bfloat16, FP32 accumulation
 * on the bf16 matrix cores, FP32 master weights trained by Adam.
 *
 * Conventions as in smm.h (status codes, ownership, the context's stream).
 * Tensor arguments documented as "device" are device pointers on the
 * context's device; the others are host memory.
 */
#ifndef SMM_CNN_H
#define SMM_CNN_H

#include <stddef.h>

#include "smm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* start mode for smm_batch_solve (and smm_solve): the network attached by
 * smm_batch_set_warmstart (smm_set_warmstart); falls back to
 * SMM_START_DIFFUSION per problem whose prediction is not finite */
#define SMM_START_LEARNED 3

typedef struct smm_cnn smm_cnn;

/* A network of n_layers 3x3 convolutions with channel counts
 * channels[0..n_layers] (each 1..64; padded internally to 16, 32 or 64) on
 * height x width images, for batches of up to max_batch images.  Weights
 * start at zero; set them with smm_cnn_set_params.  SMM_EINVAL on bad
 * sizes, SMM_ENOMEM if the device buffers do not fit. */
int smm_cnn_create(smm_ctx* ctx, int n_layers, const int* channels, int height, int width, int max_batch,
                   smm_cnn** out);
int smm_cnn_destroy(smm_cnn* net);
/* Number of parameters: for each layer l, W[c_{l+1}][c_l][3][3] followed by
 * b[c_{l+1}] (FP32, this order, layer after layer). */
int smm_cnn_num_params(const smm_cnn* net, size_t* n);
/* Copy n = smm_cnn_num_params floats (host) into the master weights and
 * reset the Adam moments and step count. */
int smm_cnn_set_params(smm_cnn* net, const float* params, size_t n);
int smm_cnn_get_params(smm_cnn* net, float* params, size_t n);
/* y = net(x).  x: device [batch][height][width][channels[0]] FP32 (rounded
 * to bf16 on entry); y: device [batch][height][width][channels[n_layers]]
 * FP32.  batch <= max_batch.  Queued on the context's stream. */
int smm_cnn_forward(smm_cnn* net, const float* x, int batch, float* y);
/* One forward and backward pass of the weighted mean squared error
 *     loss = mean over (b, pixel, o) of w_o (y - t)^2
 * over the images idx[0..batch) of x_all (device, n_all images, layout of
 * x) against targets t_all (device, n_all images, layout of y).  idx:
 * device int array, or NULL for images 0..batch-1; an index outside
 * [0, n_all) makes the call return SMM_EINVAL.  chan_weight: host [channels[n_layers]] or NULL (all 1).
 * The parameter gradient stays in the network for smm_cnn_adam_step; grad
 * (host, nullable) receives a copy in the smm_cnn_num_params layout.  loss
 * (host, nullable) receives the loss.  Synchronises the stream. */
int smm_cnn_loss_grad(smm_cnn* net, const float* x_all, const float* t_all, int n_all, const int* idx, int batch,
                      const float* chan_weight, double* loss, float* grad);
/* One Adam step (Kingma and Ba, 2015) on the FP32 master weights with the
 * gradient of the last smm_cnn_loss_grad, then the bf16 weight copies are
 * refreshed.  SMM_ESTATE if no gradient is held. */
int smm_cnn_adam_step(smm_cnn* net, float lr, float beta1, float beta2, float eps);

/* ---------------------------------------------------------------------------
 * Warm start of a batch.  Every problem of the batch must be an nx x ny
 * Cartesian problem of one order p (the network's height = ny, width = nx).
 * Features per element (channels): log10 sigma_t, sigma_s / sigma_t, element
 * mean of q, distance of the element centre to the boundary, log10 of the
 * diffusion-start flux scale s_K (element mean of |varphi_D|) minus its
 * problem mean, and the (p+1)^2 nodal values varphi_D / s_K - 1.
 * Targets per element: (p+1)^2 values (varphi - varphi_D) / s_K, then
 * (p+1)^2 values of the correction source b - b_fixed divided by
 * (h_x h_y s_K).
 * ------------------------------------------------------------------------- */
/* Number of feature and target channels for the batch's order. */
int smm_batch_warmstart_dims(const smm_batch* batch, int* n_features, int* n_targets, int* height, int* width);
/* Solve the diffusion start (zero correction source) of every problem to
 * inner_tol and keep it as varphi_D. */
int smm_batch_diffusion(smm_batch* batch, double inner_tol, int max_inner);
/* features: device [count][ny][nx][n_features] FP32 for problems
 * first..first+count-1 (needs smm_batch_diffusion). */
int smm_batch_warmstart_features(smm_batch* batch, int first, int count, float* features);
/* targets: device [count][ny][nx][n_targets] FP32 from the last
 * smm_batch_solve (needs smm_batch_diffusion before it). */
int smm_batch_warmstart_targets(smm_batch* batch, int first, int count, float* targets);
/* Attach (or detach with NULL) the network used by SMM_START_LEARNED.  Its
 * input and output channel counts must match smm_batch_warmstart_dims.  The
 * network must outlive its use by the batch. */
int smm_batch_set_warmstart(smm_batch* batch, smm_cnn* net);
/* The same network for smm_solve on one problem (SMM_START_LEARNED), which
 * runs as a batch of one: the problem must be a uniform Cartesian mesh with
 * an isotropic source, and the network must match it (height ny, width nx,
 * the channel counts of smm_batch_warmstart_dims).  NULL detaches it.  The
 * network must outlive its use by the problem. */
int smm_set_warmstart(smm_problem* prob, smm_cnn* net);
/* After a solve with SMM_START_LEARNED: used[k] = 1 if problem k started
 * from the learned start, 0 if it fell back to the diffusion start (non-finite
 * prediction). */
int smm_batch_warmstart_used(const smm_batch* batch, int* used);

#ifdef __cplusplus
}
#endif

#endif /* SMM_CNN_H */
