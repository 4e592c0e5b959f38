/*
 * warmstart.h -- C ABI of the learned initial trajectory for the iterated
 * smoother (MI355X, gfx950, FP32).
 *
 * Every iteration of the iterated smoother (Section 3) linearises around the
 * trajectory of the previous iteration, so the first iteration needs an
 * initial trajectory xbar^(0); the paper does not say how to choose it.  This
 * library proposes one with a small 1-D convolutional network that maps a
 * window of W bearing measurements to the states of those W steps.  It is
 * trained on smoother outputs (converged means of the plain method), with
 * hand-written forward, backward and Adam kernels.
 *
 * Network (one window, FP32; L = W / P positions after the patch embedding):
 *   input   x[c][t]: c = 2 s + 0 / 1 holds sin / cos of bearing s at step t
 *   embed   h0 = relu(conv(x; kernel P, stride P))                 width C
 *   hidden  h_l = h_{l-1} + relu(conv(h_{l-1}; kernel 3, dilation 2^(l-1),
 *           zero padding inside the window)),   l = 1..H
 *   head    out[u * nx + i][j] = WH h_H + bH   -> normalised state i at step
 *           P j + u; state = mu_i + sigma_i * out
 *   loss    mean of (out - (label - mu) / sigma)^2 over windows, steps, states
 *   Parameters: one flat float vector W0, b0, (W_l, b_l) for l = 1..H, WH, bH,
 *   weights [Cout][Cin][K] row-major (the head's as [P nx][C]).
 *
 * Windows of a track with T measurements: ceil(T / W) windows, window w
 * starting at step 1 + W w, the last one starting at max(1, T - W + 1) (steps
 * past T repeat y_T).  Step k takes the network's estimate from window
 * min((k - 1) / W, n_windows - 1); slot 0 (x_0) takes the estimate of step 1.
 *
 * Conventions: every call returns ws_status and never aborts across the ABI;
 * ws_last_error() explains a failure.  Device pointers (d_*) are caller-owned
 * device memory; host pointers are read during the call only.  All device work
 * is queued on the stream given to ws_create, and the caller orders other
 * streams against it.  The handle owns its parameters, optimiser state and
 * workspace.  One handle per host thread at a time.
 */
#ifndef WARMSTART_H_
#define WARMSTART_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ws_net* ws_t;

typedef enum {
  WS_OK = 0,
  WS_EINVAL = 1,   /* invalid argument, decided on the host before device work */
  WS_ENOMEM = 2,   /* device allocation failed */
  WS_EDEVICE = 3,  /* HIP runtime error */
  WS_ESTATE = 5    /* call not valid now (NULL handle, no tracks planned) */
} ws_status;

typedef struct {
  int32_t window;     /* W, measurement steps per window (64) */
  int32_t patch;      /* P, steps per patch; W % P == 0 and (W / P) % 4 == 0 (4) */
  int32_t width;      /* C, channels of the embedding and hidden layers (128) */
  int32_t hidden;     /* H, dilated residual layers, 0..12 (4) */
  int32_t nx;         /* states predicted per step (5) */
  int32_t ny;         /* bearings per step; the input has 2 ny channels (2) */
  int32_t max_batch;  /* most windows per training step; inference runs in chunks of it (1024) */
} ws_config;

typedef struct {
  float lr, beta1, beta2, eps;   /* Adam (Kingma & Ba, 2015) */
} ws_adam;

/* Defaults given in parentheses above. */
void ws_config_defaults(ws_config* cfg);

/* Number of parameters of the network that cfg describes (0 if invalid). */
int64_t ws_param_count(const ws_config* cfg);

/* Validates cfg, allocates parameters (zero), Adam state and workspace for
 * max_batch windows on the current device.  *out = NULL on failure. */
ws_status ws_create(const ws_config* cfg, void* hip_stream, ws_t* out);

/* Copies n = ws_param_count() host floats into the parameters and resets the
 * Adam moments and step count.  Waits for the copy. */
ws_status ws_set_params(ws_t h, const float* params, int64_t n);

/* Waits for the stream and copies the parameters to host params[n]. */
ws_status ws_get_params(ws_t h, float* params, int64_t n);

/* Output normalisation: state i = mu[i] + sigma[i] * out (host, nx each,
 * sigma > 0).  Defaults: mu = 0, sigma = 1. */
ws_status ws_set_normalization(ws_t h, const float* mu, const float* sigma);

/* Plans the windows of n_tracks tracks with measurement offsets offsets[0..n]
 * (host, T_i = offsets[i+1] - offsets[i] >= 1, as in smoother.h).  Used by
 * ws_windows, ws_labels and ws_trajectory.  *n_windows (nullable) receives the
 * number of windows. */
ws_status ws_set_tracks(ws_t h, const int64_t* offsets, int32_t n_tracks, int64_t* n_windows);

/* Network inputs of every planned window: d_y device double [sum T][ny]
 * (bearings, the measurements given to the smoother) -> d_x device float
 * [n_windows][2 ny][W]. */
ws_status ws_windows(ws_t h, const double* d_y, float* d_x);

/* Training labels of every planned window from smoothed means: d_mean device
 * double [sum (T + 1)][nx] (smoother_result_device layout) -> d_lab device
 * float [n_windows][W][nx]. */
ws_status ws_labels(ws_t h, const double* d_mean, float* d_lab);

/* One Adam step on the mean-squared error of windows d_idx[0..n-1] (device
 * int32, n <= max_batch) of a data set of n_data windows d_x / d_lab (layouts
 * of ws_windows / ws_labels): forward, loss, backward, update.  When loss_out
 * is not NULL the call waits and stores the batch loss before the update.
 * Indices outside [0, n_data) are device data the host cannot see: the
 * kernels read no memory for them (zero window) and the next call that waits
 * (ws_train_step with loss_out, ws_gradient, ws_predict) returns WS_EINVAL. */
ws_status ws_train_step(ws_t h, const float* d_x, const float* d_lab, int64_t n_data, const int32_t* d_idx,
                        int32_t n, const ws_adam* opt, float* loss_out);

/* Loss and gradient (no update) of the same batch: waits and copies the
 * gradient to host grad[ws_param_count()] (nullable) and the loss to
 * loss_out (nullable). */
ws_status ws_gradient(ws_t h, const float* d_x, const float* d_lab, int64_t n_data, const int32_t* d_idx,
                      int32_t n, float* grad, float* loss_out);

/* Predicted states of windows d_idx[0..n-1] of d_x (n_data windows) ->
 * d_states device float [n][W][nx] (any n; runs in chunks of max_batch);
 * waits for the stream. */
ws_status ws_predict(ws_t h, const float* d_x, int64_t n_data, const int32_t* d_idx, int32_t n, float* d_states);

/* Initial trajectory of the planned tracks straight from the measurements:
 * d_y device double [sum T][ny] -> d_mean device double [sum (T + 1)][nx],
 * the layout smoother_set_trajectory_device takes. */
ws_status ws_trajectory(ws_t h, const double* d_y, double* d_mean);

/* As ws_trajectory, with the network's matrix products on the matrix cores:
 * operands rounded to BF16 (to nearest even), FP32 accumulation, FP32 bias,
 * activations and normalisation.  The trajectory is a starting point of the
 * smoother, so the rounding only moves the start; ws_trajectory stays the
 * FP32 evaluation the network was trained with. */
ws_status ws_trajectory_mfma(ws_t h, const double* d_y, double* d_mean);

/* Message of the last failure on h (NULL: last ws_create failure on this thread). */
const char* ws_last_error(ws_t h);

/* Releases the handle and its device memory; NULL-safe. */
void ws_destroy(ws_t h);

#ifdef __cplusplus
}
#endif

#endif /* WARMSTART_H_ */
