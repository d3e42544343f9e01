/*
 * lbm_mlp.h - C ABI of the critical-pressure surrogate network (gfx950).
 *
 * The paper solves every critical pressure by simulation; this network is an
 * extension that proposes the starting bracket of the bisection (the
 * simulation still decides the result).  It maps 6 features of a channel
 * problem to one number (the log10 of the critical forcing, standardised by
 * the caller):
 *
 *   x in R^6 -> 128 -> 128 -> 128 -> 1,
 *   hidden layers z = W a + b followed by GELU(z) = z/2 (1 + erf(z / sqrt 2)),
 *   linear output, loss L = mean over the batch of (y - t)^2,
 *   Adam (Kingma & Ba 2015) with bias-corrected moments.
 *
 * Parameters are one flat FP32 vector of LBM_MLP_PARAMS values, in the order
 * W1 (128 x 6, one row per output unit), b1 (128), W2 (128 x 128), b2, W3
 * (128 x 128), b3, W4 (1 x 128), b4 (1).  All arithmetic is FP32; the 128 x 128
 * contractions run on the matrix cores, the sums over a batch accumulate in a
 * fixed order (results are deterministic).
 *
 * All pointers are device pointers unless stated otherwise; all calls enqueue
 * on hip_stream (a hipStream_t, NULL for the null stream) and return without
 * waiting, except where noted.  Status codes and lbm_last_error are those of
 * lbm.h.  The library allocates no device memory: the caller passes a
 * workspace of at least lbm_mlp_workspace_bytes(B) bytes.
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_IN 6
#define LBM_MLP_HIDDEN 128
#define LBM_MLP_PARAMS 34049

/* Workspace bytes for batches of up to max_batch samples (activations and
 * deltas of every sample, per-block loss partials); 0 if max_batch < 1. */
size_t lbm_mlp_workspace_bytes(int32_t max_batch);

/* y[B] = net(params, X[B][6]) (row-major X).  Keeps the activations in ws for
 * a following lbm_mlp_backward on the same X.  1 <= B <= the ws capacity. */
lbm_status lbm_mlp_forward(const float* params, const float* X, int32_t B, float* y, void* ws,
                           size_t ws_bytes, void* hip_stream);

/* Gradient of L = mean_b (y_b - t_b)^2 with respect to the parameters, for
 * the y and activations left in ws by lbm_mlp_forward(params, X, B, y, ws):
 * grad[LBM_MLP_PARAMS] is overwritten; loss (one float, may be NULL) receives
 * L. */
lbm_status lbm_mlp_backward(const float* params, const float* X, const float* y,
                            const float* t, int32_t B, float* grad, float* loss, void* ws,
                            size_t ws_bytes, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): lbm_mlp_forward followed by lbm_mlp_backward on the same batch,
 * with the activations and deltas kept in a fixed device array of the
 * library instead of a caller workspace.  Writes y[B], grad[LBM_MLP_PARAMS]
 * and (if not NULL) loss[0], bit for bit as the two calls would with a
 * workspace.  1 <= B <= LBM_MLP_NOALLOC_MAX_BATCH, else LBM_ERR_INVALID.
 * The array holds 9 x 2048 x 128 + 128 floats (9.4 MB); each device the
 * library runs on keeps its own copy until the process ends, and every call
 * on a device shares it: calls that overlap on one device (two streams, two
 * threads) race and their results are undefined.  Allocates nothing; the
 * first call on a device looks up that device's copy (no allocation either).
 */
#define LBM_MLP_NOALLOC_MAX_BATCH 2048
lbm_status lbm_mlp_gradient_noalloc(const float* params, const float* X, const float* t,
                                    int32_t B, float* y, float* grad, float* loss,
                                    void* hip_stream);

/* One Adam step k >= 1 on params, in place, with first / second moment
 * vectors m, v (LBM_MLP_PARAMS each, zero before step 1). */
lbm_status lbm_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t k,
                        float lr, float beta1, float beta2, float eps, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_MLP_H */
