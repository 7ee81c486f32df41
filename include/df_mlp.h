/*
 * df_mlp.h - C ABI of the learned warm start: a small multilayer perceptron
 * trained and evaluated by hand-written FP32 matrix-core kernels (libdf.so).
 *
 * The network maps per-(instance, k) features to the dual self-energy
 * Sigma~(k, nu) at the positive fermionic frequencies; its prediction is only
 * a starting point of df_iterate, which still runs to the same tolerance, so
 * results do not depend on it (only the iteration count does).
 *
 * Network: n_layers affine layers with dims[0] -> dims[1] -> ... ->
 * dims[n_layers]; SiLU after every layer but the last.
 * Parameters: one FP32 device buffer, layer by layer: W_l (dims[l+1] x dims[l],
 * row-major) then b_l (dims[l+1]).  Inputs X are row-major [batch][dims[0]],
 * outputs and targets [batch][dims[n_layers]].
 *
 * Loss: mean squared error over all batch x dims[n_layers] outputs.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
 *
 * All pointers are device pointers except dims (host).  The caller owns every
 * buffer and the workspace (size from df_mlp_workspace_size, 256-byte
 * aligned).  Calls are asynchronous on the given stream and return the
 * status codes of df.h.  Reductions run in a fixed order: results are
 * reproducible bit for bit.
 */
#ifndef DF_MLP_H
#define DF_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "df.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DF_MLP_MAX_LAYERS 8
#define DF_MLP_MAX_WIDTH 1024

/* Number of FP32 parameters of the network. */
int df_mlp_param_count(int32_t n_layers, const int32_t *dims, size_t *count);

/* Workspace bytes for a batch of `batch` rows (forward and training). */
int df_mlp_workspace_size(int32_t n_layers, const int32_t *dims, int32_t batch, size_t *bytes);

/* Y = network(X). */
int df_mlp_forward(int32_t n_layers, const int32_t *dims, const float *params, const float *X,
                   int32_t batch, float *Y, void *ws, size_t ws_bytes, df_stream_t stream);

/* loss (device scalar, may be NULL) and grads (same layout as params) of the
 * mean squared error of network(X) against T. */
int df_mlp_loss_grad(int32_t n_layers, const int32_t *dims, const float *params, const float *X,
                     const float *T, int32_t batch, float *grads, float *loss, void *ws,
                     size_t ws_bytes, df_stream_t stream);

/* One Adam update of params from grads; m, v are the moment buffers (zero at
 * step 1), step counts from 1, lr is the learning rate. */
int df_mlp_adam(size_t count, float *params, const float *grads, float *m, float *v, int32_t step,
                float lr, df_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DF_MLP_H */
