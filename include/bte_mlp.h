/* Learned warm start for the superlattice BTE sweep: a small multilayer
 * perceptron that maps an instance's parameters (E_dc, E_w, omega, B, mu) to
 * a compressed periodic steady state, so the solver can start near the
 * attractor instead of from f0 (the periodic regime the absorption of
 * Eq. (absorption_def) is averaged over, Sec. 2).  The network is not part of
 * the paper's method; the solver still runs to its own convergence test.
 *
 * Network: 5 -> 256 -> 256 -> 8192, GELU (erf form) after both hidden
 * layers, no activation on the output.  Parameters: 2,172,672 FP32 master
 * values in one flat array, in this order and layout (row-major, [out][in]):
 *     W1 [256][5], b1 [256], W2 [256][256], b2 [256], W3 [8192][256], b3 [8192].
 * The two large layers run on the matrix cores with BF16 operands (weights and
 * activations rounded to BF16, FP32 accumulation), or with FP32 operands in
 * the FP32 precision mode; the first layer (5 inputs) runs in FP32 on the
 * vector ALUs.  Training uses Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the
 * FP32 master values.
 *
 * Inputs are normalised per feature, x_i' = (x_i - shift_i) / scale_i, and the
 * regression target is the coefficient array times out_scale.  The 64 x 128
 * coefficient layout is the one bte_batch_set_warm_start reads and
 * bte_batch_set_state_output writes (include/bte.h).  The loss is the mean of
 * squared differences over the batch's n x 8192 scaled targets.
 *
 * Memory: the caller allocates the device workspace (bte_mlp_workspace_bytes)
 * and keeps it alive until bte_mlp_destroy; the library never allocates
 * device memory.  Every call queues work on the handle's stream and returns
 * without a host synchronisation, except bte_mlp_get_normalization.  Device
 * arrays passed to a call must stay valid until the work queued by that call
 * has completed.  A handle is not thread-safe.  Errors are returned as
 * bte_status codes with a message in bte_last_error().
 */
#ifndef BTE_MLP_H
#define BTE_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "bte.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { BTE_MLP_IN = 5, BTE_MLP_HIDDEN = 256, BTE_MLP_OUT = 8192 };

typedef enum { BTE_MLP_BF16 = 0, BTE_MLP_FP32 = 1 } bte_mlp_precision;

typedef struct bte_mlp bte_mlp;

/* Number of FP32 master parameters (2,172,672). */
int64_t bte_mlp_param_count(void);

/* Device workspace for batches of up to max_batch rows (training and
 * gradient calls; inference processes larger inputs in chunks of this size).
 * Returns 0 for max_batch < 1 or an unknown precision. */
size_t bte_mlp_workspace_bytes(int32_t max_batch, int32_t precision);

/* Create a network on the caller's workspace.  The parameters start at zero
 * and the normalisation at the identity (shift 0, scale 1, out_scale 1): call
 * bte_mlp_set_params and bte_mlp_fit_normalization (or _set_normalization)
 * before use.  hip_stream: a hipStream_t or NULL (default stream). */
bte_status bte_mlp_create(int32_t max_batch, int32_t precision, void* workspace,
                          size_t workspace_bytes, void* hip_stream, bte_mlp** out);

/* Replace the FP32 master parameters (device array of bte_mlp_param_count()
 * floats, layout above), refresh the matrix-core copies and reset Adam's
 * moments and step count. */
bte_status bte_mlp_set_params(bte_mlp* h, const float* dev_params);

/* Copy the FP32 master parameters to a device array of param_count floats. */
bte_status bte_mlp_get_params(bte_mlp* h, float* dev_params);

/* Fit the normalisation on a data set of n rows: shift_i and scale_i are the
 * mean and standard deviation (population form) of feature i, with scale 1
 * for a feature whose deviation is below 1e-6 (1 + |mean|); out_scale is
 * 1 / sqrt(mean of the squared coefficients), 1 when that mean is 0.
 * dev_features: n x 5 floats (E_dc, E_w, omega, B, mu); dev_coeffs: n x 8192
 * floats. */
bte_status bte_mlp_fit_normalization(bte_mlp* h, const float* dev_features,
                                     const float* dev_coeffs, int32_t n);

/* Host copies of the normalisation: 11 floats, shift[5], scale[5], out_scale.
 * _get synchronises the stream. */
bte_status bte_mlp_get_normalization(bte_mlp* h, float* host11);
bte_status bte_mlp_set_normalization(bte_mlp* h, const float* host11);

/* Predicted coefficients for n rows of features: dev_coeffs receives
 * n x 8192 floats in the warm-start layout (unscaled: prediction/out_scale). */
bte_status bte_mlp_forward(bte_mlp* h, const float* dev_features, int32_t n, float* dev_coeffs);

/* Loss and its gradient for a batch of n rows of a data set of n_rows rows
 * (dev_features: n_rows x 5, dev_coeffs: n_rows x 8192), without changing
 * the parameters.  The batch is rows dev_index[0..n-1] (n int32 values), or
 * rows 0..n-1 when dev_index is NULL (then n <= n_rows).  n <= max_batch.  An
 * index outside 0..n_rows-1 is not read: its row enters as a zero-gradient
 * row (the loss still divides by n).  dev_grad: param_count floats (layout of
 * the parameters) or NULL; dev_loss: 1 float or NULL. */
bte_status bte_mlp_loss_grad(bte_mlp* h, const float* dev_features, const float* dev_coeffs,
                             int32_t n_rows, const int32_t* dev_index, int32_t n,
                             float* dev_grad, float* dev_loss);

/* One Adam step with learning rate lr on a batch (as bte_mlp_loss_grad);
 * dev_loss (1 float or NULL) receives the loss before the step. */
bte_status bte_mlp_train_step(bte_mlp* h, const float* dev_features, const float* dev_coeffs,
                              int32_t n_rows, const int32_t* dev_index, int32_t n, float lr,
                              float* dev_loss);

void bte_mlp_destroy(bte_mlp* h);

#ifdef __cplusplus
}
#endif

#endif /* BTE_MLP_H */
