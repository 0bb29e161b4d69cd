/* Learned warm start for the implicit CP-ALS step (libcpals, gfx950).
 *
 * The implicit step of Section 3.1 minimises ||A f_{n+1} - B f_n|| by alternating least
 * squares started from a guess of f_{n+1}; the plain method starts from f_n.  This part of
 * the library predicts a better guess, factor column by factor column: the linear
 * extrapolation of the column in time plus a correction from a small 1-D convolutional
 * network.  The caller then runs cp_als_step from it (ALS refines the guess to the same
 * tolerance and stays the arbiter of the result).
 *
 * Network (one sample = column l of the factor of dimension k, n = n_k grid points):
 *   input   x[3][n] = (U_k(t_{n-1})[:, l] / s, U_k(t_n)[:, l] / s, c_k),  s = rms(U_k(t_n)[:, l])
 *           (s = 1 for an all-zero column), c_k a per-dimension scalar supplied by the caller;
 *   layers  four circular convolutions of width 5 over the periodic grid,
 *           z[o][i] = b[o] + sum_{c,t} W[o][c][t] x[c][(i + t - 2) mod n],
 *           channels 3 -> 32 -> 32 -> 32 -> 1, ReLU after the first three;
 *   output  y[n]; the guess is 2 U_k(t_n)[:, l] - U_k(t_{n-1})[:, l] + 2^-12 s y (a zero network
 *           gives the linear extrapolation), the training target
 *           (U_k(t_{n+1}) - 2 U_k(t_n) + U_k(t_{n-1}))[:, l] / (2^-12 s); the fixed power-of-two
 *           output scale lets the network produce the small correction as outputs of order one;
 *   loss    mean squared error over samples and grid points; Adam (0.9, 0.999, 1e-8).
 * Parameters in natural order: for each layer W[o][c][t] (row-major) then b[o]; 10977 in all.
 * Precision: BF16 weights, activations and gradients, FP32 accumulation on the matrix
 * cores, FP32 master weights and moments.
 *
 * Memory: the network object owns its device memory (weights, moments, activation and
 * gradient buffers for up to max_batch samples of n points).  All pointers named *_dev are
 * device memory owned by the caller; *_host are host memory.  Calls are asynchronous on the
 * handle's stream except where a host output is returned (the call then synchronises).
 * Errors: CP_ERR_INVALID_ARG for null or out-of-range arguments, CP_ERR_SHAPE for sizes
 * beyond the object's capacity, CP_ERR_UNSUPPORTED for grids the kernels do not tile
 * (n must be a multiple of 16; n <= 1024 for prediction, n <= 256 for training),
 * CP_ERR_HIP for a failed runtime call (cp_last_error has the message).
 */
#ifndef CPALS_WS_H
#define CPALS_WS_H

#include "cpals.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cp_ws_net_s* cp_ws_net;

/* Number of parameters (10977). */
int32_t cp_ws_num_params(void);

/* Create a network for grids of n points and batches of up to max_batch samples, with
 * FP32 master parameters params_host (natural order, cp_ws_num_params() values). */
cp_status cp_ws_create(cp_handle h, const float* params_host, int32_t n, int32_t max_batch, cp_ws_net* net);
cp_status cp_ws_destroy(cp_ws_net net);

/* Copy the FP32 master parameters to params_host (synchronises). */
cp_status cp_ws_get_params(cp_handle h, cp_ws_net net, float* params_host);

/* Network output y_dev[B][n] (FP32) for inputs x_dev[B][3][n] (FP32, natural layout). */
cp_status cp_ws_forward(cp_handle h, cp_ws_net net, const float* x_dev, int32_t B, float* y_dev);

/* Gradient of the loss with respect to the parameters (grad_dev, natural order, FP32) for
 * inputs x_dev[B][3][n] and targets target_dev[B][n]; the loss is written to *loss_host. */
cp_status cp_ws_gradients(cp_handle h, cp_ws_net net, const float* x_dev, const float* target_dev, int32_t B,
                          float* grad_dev, float* loss_host);

/* One Adam step on B samples of a trajectory.  traj_dev holds T time levels of C columns of
 * n points each ([T][C][n], FP64: for a CP trajectory, the concatenated factor panels of every
 * step); sample j is (t, c) = (samples_host[2j], samples_host[2j+1]) with 1 <= t <= T - 2,
 * using columns (t-1, t, t+1); coef_host[c] is the scalar channel of column c.  The loss
 * before the step is written to *loss_host. */
cp_status cp_ws_train_step(cp_handle h, cp_ws_net net, const double* traj_dev, int32_t T, int32_t C,
                           const int32_t* samples_host, const double* coef_host, int32_t B, float lr, float* loss_host);

/* Predicted next factors: f_guess column (k, l) = 2 f_cur column - f_prev column + 2^-12 s y
 * for the inputs built from f_prev and f_cur; coef_host[k] per dimension; f_guess may be
 * f_cur.
 * All three tensors have the same d, n_k and rank; every n_k must equal the network's n;
 * d * r <= max_batch. */
cp_status cp_ws_predict(cp_handle h, cp_ws_net net, const cp_tensor* f_prev, const cp_tensor* f_cur,
                        const double* coef_host, cp_tensor* f_guess);

#ifdef __cplusplus
}
#endif

#endif /* CPALS_WS_H */
