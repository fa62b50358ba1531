/*
 * qp_mlp.h -- C-ABI of the learned warm start for the MI355X rAPDHG solver.
 *
 * The paper's Algorithm 1 takes an initial point (x^{0,0}, y^{0,0}) as input and
 * Theorem 1 bounds the work by dist(z^{0,0}, Z*): a better initial point means
 * fewer iterations.  This library provides a small multilayer perceptron that
 * maps the varying data of a parametrised QP family to a starting point and a
 * primal weight; it is trained on solutions the solver itself produced.  The
 * solver's own KKT test (qp_solve / qp_batch_solve with warm_fallback = 1)
 * checks every prediction, and a cold start is used whenever the prediction is
 * worse.
 *
 * Network: sizes[0] -> sizes[1] -> ... -> sizes[L], ReLU after every hidden
 * layer, linear output.  Compute: BF16 operands on the MFMA matrix cores with
 * FP32 accumulation; FP32 master weights, FP32 gradients, FP32 Adam state.
 * Loss: mean squared error over all outputs of the batch.
 *
 * Parameter vector order (host arrays of qp_mlp_num_params floats): for each
 * layer l = 0..L-1, the weight W_l (sizes[l+1] x sizes[l], row-major: one row per
 * output unit), then the bias b_l (sizes[l+1]).
 *
 * Device arrays: x, out and target are FP32, row-major, one row per sample,
 * in device memory; calls are ordered on the handle's own stream and return
 * after it completes.  Errors: QP_ERR_* codes from qp.h; qp_last_error() gives
 * the message.
 */
#ifndef QP_MLP_MI355X_H
#define QP_MLP_MI355X_H

#include <stdint.h>

#include "qp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qp_mlp qp_mlp;

/* n_layers >= 1 linear layers; sizes has n_layers + 1 entries (all >= 1);
 * max_batch >= 1 bounds the batch of every later call.  Weights start at zero;
 * load them with qp_mlp_set_params. */
int qp_mlp_create(int32_t n_layers, const int32_t *sizes, int32_t max_batch, int32_t device,
                  qp_mlp **out);
void qp_mlp_free(qp_mlp *h);
int64_t qp_mlp_num_params(const qp_mlp *h);
/* host FP32 arrays of qp_mlp_num_params entries */
int qp_mlp_set_params(qp_mlp *h, const float *params);
int qp_mlp_get_params(qp_mlp *h, float *params);
int qp_mlp_get_grads(qp_mlp *h, float *grads);
/* replaces the gradient with a host FP32 array of qp_mlp_num_params entries (for
 * example gradients summed over several replicas); a following qp_mlp_adam_step
 * applies it. */
int qp_mlp_set_grads(qp_mlp *h, const float *grads);

/* out[batch x sizes[L]] = network(x[batch x sizes[0]]); keeps the activations
 * for a following qp_mlp_backward. */
int qp_mlp_forward(qp_mlp *h, const float *x, int32_t batch, float *out);
/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): the inference part of
 * qp_mlp_forward with every temporary (BF16 activations, split-K partial tiles) in a
 * fixed workspace of QP_MLP_NOALLOC_SCRATCH_BYTES that the library holds in static
 * device memory, one per GPU until the process ends, located by qp_mlp_create; the
 * call allocates nothing.  out[batch x sizes[L]] (device, FP32) receives the values
 * qp_mlp_forward returns for the same x.  The activations are not kept (no
 * qp_mlp_backward may rely on this call) and no buffer of the handle is written.
 * Every call on one GPU shares its workspace, which keeps the last call's contents:
 * calls that overlap in time on the same GPU (from other threads or handles) race,
 * and the caller must serialise them.  A batch whose workspace would exceed the limit
 * (2 x batch x the widest padded layer input in BF16, plus the split-K partials) is
 * rejected with QP_ERR_INVALID_ARGUMENT before any device work.  Blocking on the
 * handle's stream, like qp_mlp_forward. */
#define QP_MLP_NOALLOC_SCRATCH_BYTES (32u << 20)
int qp_mlp_forward_noalloc(qp_mlp *h, const float *x, int32_t batch, float *out);
/* gradient of the mean squared error against target[batch x sizes[L]] at the
 * activations of the last forward call (same batch); *loss receives the loss. */
int qp_mlp_backward(qp_mlp *h, const float *target, int32_t batch, float *loss);
/* Minibatch forms for training on a data set resident in device memory: x_all
 * [n_rows x sizes[0]] and target_all [n_rows x sizes[L]] (device, FP32, row-major)
 * hold every sample, and rows (device, int32, batch entries) names the samples of
 * the minibatch: sample i is row rows[i].  The rows are gathered by the kernels that
 * read the data (BF16 conversion of the input, the loss gradient), so no copy of the
 * minibatch is made.  An index outside [0, n_rows) yields QP_ERR_INVALID_ARGUMENT
 * after the call (that sample is read as zeros); qp_mlp_backward_rows must follow a
 * qp_mlp_forward_rows (or qp_mlp_forward) of the same batch size, and its rows should
 * be the ones that forward used. */
int qp_mlp_forward_rows(qp_mlp *h, const float *x_all, int64_t n_rows, const int32_t *rows,
                        int32_t batch, float *out);
int qp_mlp_backward_rows(qp_mlp *h, const float *target_all, int64_t n_rows,
                         const int32_t *rows, int32_t batch, float *loss);
/* one Adam step (bias-corrected, step >= 1) on every parameter with the current
 * gradients; refreshes the BF16 copies used by forward. */
int qp_mlp_adam_step(qp_mlp *h, float lr, float beta1, float beta2, float eps, int32_t step);

#ifdef __cplusplus
}
#endif
#endif
