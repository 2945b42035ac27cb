/*
 * srg.h -- C ABI of the outcome/trajectory surrogate of the drop-particle runs.
 *
 * A multilayer perceptron 6 -> 256 -> 256 -> 256 -> 256 -> 51 (ReLU between
 * layers) maps the six parameters of a run -- sliding and rolling friction
 * coefficients, drop radius, drop body force, particle contact angle, particle
 * radius (the quantities the section on particle removal varies) -- to three
 * outcome logits (picked up / pushed / left behind) and the particle's
 * displacement at 16 times (48 values).  Inputs and trajectory targets are
 * standardised by the caller.
 *
 * Training and inference run on the GPU in BF16 matrix-core (MFMA) kernels with
 * FP32 accumulation; master weights, gradients and the Adam state are FP32.
 * Loss: mean softmax cross-entropy of the logits + w_traj * mean squared error
 * of the 48 trajectory outputs.
 *
 * Conventions: returns 0 or a negative status (the lbm_status codes of lbm.h);
 * errors are sticky per context.  The caller owns the device workspace (256-byte
 * aligned, srg_workspace_bytes long) and every host buffer.  Parameters travel
 * as FP32 in the canonical order W1 (6x256, row-major in x out), b1 (256), W2,
 * b2, W3, b3, W4, b4 (256x256, 256), W5 (256x51), b5 (51): SRG_PARAMS floats.
 */
#ifndef SRG_H
#define SRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRG_IN 6
#define SRG_OUT 51
#define SRG_PARAMS 212275

typedef struct srg_ctx srg_ctx;

/* Workspace for batches of up to max_batch samples (a multiple of 64) and a
 * training set of up to max_train samples.  0 if an argument is invalid. */
size_t srg_workspace_bytes(int32_t max_batch, int32_t max_train);

/* Create a context on the caller's workspace and stream (hipStream_t, NULL for
 * the null stream).  Parameters start at zero: set them with srg_set_params. */
int srg_create(void* dev_workspace, size_t ws_bytes, int32_t max_batch, int32_t max_train,
               void* hip_stream, srg_ctx** out);

/* Set all parameters (host, SRG_PARAMS floats, canonical order) and reset the
 * optimiser state; get them back. */
int srg_set_params(srg_ctx* ctx, const float* params);
int srg_get_params(srg_ctx* ctx, float* params);

/* Upload a training set: X n x 6, label n (0 picked up, 1 pushed, 2 left
 * behind), traj n x 48 (host arrays; n <= max_train). */
int srg_set_train(srg_ctx* ctx, const float* X, const int32_t* label, const float* traj, int32_t n);

/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8) for `epochs` passes over the
 * training set in shuffled minibatches of `batch` samples (a multiple of 64, at
 * most max_batch and the set size; a final partial batch is dropped).  The
 * shuffle is a permutation drawn from `seed`.  epoch_loss (nullable, host,
 * `epochs` floats) receives each epoch's mean minibatch loss. */
int srg_train(srg_ctx* ctx, int32_t epochs, int32_t batch, float lr, float w_traj, uint64_t seed,
              float* epoch_loss);

/* One forward and backward pass over n samples (n a multiple of 64, at most
 * max_batch) without an update: gradients in the canonical order (host,
 * SRG_PARAMS floats) and the loss. */
int srg_gradients(srg_ctx* ctx, const float* X, const int32_t* label, const float* traj, int32_t n,
                  float w_traj, float* grads, float* loss);

/* Outputs y (n x 51: 3 logits, then 48 trajectory values) for inputs X (n x 6).
 * X and y are host memory, or device memory when src_is_device / dst_is_device
 * (device pointers on the context's device).  Any n >= 1; processed in chunks of
 * max_batch.  Asynchronous on the stream when both are device buffers, else
 * synchronous. */
int srg_predict(srg_ctx* ctx, const float* X, int32_t n, float* y, int32_t src_is_device,
                int32_t dst_is_device);

int srg_sync(srg_ctx* ctx);
void srg_destroy(srg_ctx* ctx);
const char* srg_last_error(const srg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SRG_H */
