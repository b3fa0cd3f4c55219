/*
 * tn_mlp.h -- C ABI of the learned sketch-size selector's regressor: a 3-layer
 * perceptron x (d_in) -> tanh(W1 x + b1) (H) -> tanh(W2 h1 + b2) (H) -> W3 h2 + b3
 * in FP32, trained with mean squared error and Adam by the library's own HIP
 * kernels.  It predicts the log input-relative variance
 * log(Var(y_hat) / prod_k ||X_k||_F^2) of one sketch estimate (the quantity the
 * variance bounds of Lemmas 6 and 9 control) from network features, so that a
 * caller can choose the sketch size m and sample count S for a target error.
 *
 * Parameters are one FP32 vector laid out as
 *   W1 [H][d_in] row-major, b1 [H], W2 [H][H] row-major, b2 [H], W3 [H], b3 [1]
 * (n_params = H d_in + H + H H + H + H + 1).  Tensors passed to these calls are
 * DEVICE pointers unless stated; work is queued on `stream` (a hipStream_t).
 * Return codes are those of tn_sketch.h (TN_OK or a negative TN_ERR_*); the
 * message is in tn_last_error().  Calls on one tn_mlp must not overlap.
 */
#ifndef TN_MLP_H
#define TN_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_mlp tn_mlp;

/* Create a network with d_in inputs (1..256) and H hidden units (1..128),
 * parameters drawn Glorot-uniform from a SplitMix64 stream keyed by seed, biases
 * zero, Adam moments zero.  A block keeps all parameters and the activations of
 * 64 rows in LDS: 4 (n_params + 64 d_in + 256 H + 66) bytes, which must leave 1 KiB
 * of the device's per-block LDS free (160 KiB on gfx950: d_in 20 with H 64 takes
 * 93 KB; H 96 allows d_in up to 40), else TN_ERR_UNSUPPORTED.
 * Errors: TN_ERR_ARG, TN_ERR_OOM, TN_ERR_HIP, TN_ERR_UNSUPPORTED. */
int tn_mlp_create(int32_t d_in, int32_t hidden, uint64_t seed, tn_mlp **out);

/* Number of parameters. */
int64_t tn_mlp_num_params(const tn_mlp *net);

/* Input width and hidden units of a network. */
int tn_mlp_shape(const tn_mlp *net, int32_t *d_in, int32_t *hidden);

/* Copy the parameter vector to / from HOST memory (n_params floats).  set
 * also clears the Adam moments and step counter. */
int tn_mlp_get_params(const tn_mlp *net, float *host_out);
int tn_mlp_set_params(tn_mlp *net, const float *host_in);

/* Predictions for n rows of X (DEVICE, n x d_in FP32 row-major) into out
 * (DEVICE, n FP32).  n = 0 does nothing (X and out may then be NULL). */
int tn_mlp_predict(tn_mlp *net, const float *X, int64_t n, void *stream, float *out);

/* Loss 0.5 mean((f(X) - y)^2) over n rows and its gradient with respect to the
 * parameters: grad (DEVICE, n_params FP32), loss (HOST, may be NULL; waits for
 * the stream). */
int tn_mlp_grad(tn_mlp *net, const float *X, const float *y, int64_t n, void *stream,
                float *grad, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * gradient of the rows [0, n) of X, y. */
int tn_mlp_step(tn_mlp *net, const float *X, const float *y, int64_t n, float lr, void *stream);

/* Train for `epochs` passes over n rows in consecutive mini-batches of `batch`
 * rows (the caller shuffles), one Adam step per batch.  losses (HOST, may be
 * NULL) receives the mean training loss of each epoch (waits for the stream). */
int tn_mlp_train(tn_mlp *net, const float *X, const float *y, int64_t n, int32_t batch,
                 int32_t epochs, float lr, void *stream, double *losses);

void tn_mlp_destroy(tn_mlp *net);

/* Save the parameters (and n_meta <= 64 caller values, e.g. the label mean,
 * standard deviation and margin of a selector) to a file: the 8 bytes
 * "TNMLP\0\0\1", then little-endian uint32 version (1), int32 d_in, int32
 * hidden, int32 n_meta, int64 n_params, n_meta doubles, n_params floats, and
 * the CRC-32 (ISO 3309 / ITU-T V.42) of every preceding byte. */
int tn_mlp_save(const tn_mlp *net, const char *path, const double *meta, int32_t n_meta);

/* Load a file written by tn_mlp_save into a new network on the current
 * device (Adam moments zero); meta receives its n_meta values (max_meta room).
 * TN_ERR_ARG for a missing file, a wrong magic or version, a size that does
 * not match the header, or a CRC mismatch. */
int tn_mlp_load(const char *path, tn_mlp **out, double *meta, int32_t max_meta, int32_t *n_meta);

/* Register the regressor that TN_SIZE_LEARNED sizing uses (tn_sketch_size,
 * tn_sketch_plan with TN_FLAG_SIZE_LEARNED): it predicts the standardized
 * label, and log v(m) = prediction * sd + mu + margin.  The network must stay
 * alive while registered; NULL unregisters.  Process-wide. */
int tn_set_size_selector(const tn_mlp *net, double mu, double sd, double margin);

#ifdef __cplusplus
}
#endif

#endif /* TN_MLP_H */
