/*
 * hrlb_mlp.h -- C ABI of the warm-start network of libhrlb: a fully connected network that
 * maps the parameters of a Couette instance and a node position to the steady profiles
 * at that node, trained and evaluated by the library's own gfx950 kernels.
 *
 * Network: 5 -> 256 -> 256 -> 256 -> 8, silu(z) = z / (1 + exp(-z)) after each hidden
 * layer, linear output.  Inputs per node (raw): log10 kn, u_w, omega, Pr, x / (L/2).
 * Outputs per node (raw): n, u_y, T, P_xx, P_xy, P_yy, q_x, q_y of the steady state.
 * The network works on standardised values, (x - mean) / std per input column and per
 * output channel, with the 26 constants given by the caller (h_norm: 5 input means,
 * 5 input stds, 8 output means, 8 output stds).
 *
 * Precision: fp32 master weights and AdamW moments; every matrix product multiplies
 * bfloat16 operands (weights, inputs, hidden activations, backward signals) on the matrix
 * cores with fp32 accumulation; biases, pre-activations, outputs, loss and gradients are
 * fp32.  Loss: mean of squared standardised errors over rows and channels.  Optimiser:
 * AdamW (beta1 0.9, beta2 0.999, eps 1e-8, decoupled weight decay on every parameter).
 *
 * Flat parameter layout (fp32, HRLB_MLP_NPARAMS values): W0[256][5], b0[256],
 * W1[256][256], b1[256], W2[256][256], b2[256], W3[8][256], b3[8]; W_l[out][in].
 *
 * Conventions are those of hrlb.h: status codes HRLB_*, hrlb_last_error(), caller-owned
 * device buffers, work enqueued on the caller's stream (no call synchronises it unless
 * stated).  Rows of inputs and targets are fp32 [rows][5] and [rows][8], row-major.
 */
#ifndef HRLB_MLP_H
#define HRLB_MLP_H

#include <stddef.h>

#include "hrlb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HRLB_MLP_IN 5
#define HRLB_MLP_OUT 8
#define HRLB_MLP_WIDTH 256
#define HRLB_MLP_NPARAMS 135176
#define HRLB_MLP_NORM 26

typedef struct hrlb_mlp hrlb_mlp;

/* Bytes of the caller's state buffer (weights, AdamW moments, constants) and work buffer
 * (activations for up to max_rows rows per call).  Errors: HRLB_EINVAL (max_rows < 1 or
 * above 2^22, NULL pointers). */
int hrlb_mlp_bytes(int max_rows, size_t* state_bytes, size_t* work_bytes);

/* Create a network on caller buffers (256-byte aligned, sizes from hrlb_mlp_bytes).
 * d_params (device, flat layout) gives the initial weights; if NULL every W_l and b_l is
 * drawn uniform in (-1/sqrt(fan_in), 1/sqrt(fan_in)) from splitmix64 of (seed, index).
 * h_norm: the 26 standardisation constants (host; stds must be > 0).  AdamW starts at
 * step 0 with zero moments.  Errors: HRLB_EINVAL, HRLB_ENOMEM, HRLB_EHIP. */
int hrlb_mlp_create(void* d_state, size_t state_bytes, void* d_work, size_t work_bytes, int max_rows,
                    const float* d_params, unsigned long long seed, const float* h_norm, void* stream,
                    hrlb_mlp** out);

/* Replace the weights (device, flat layout) and restart AdamW; copy them out. */
int hrlb_mlp_set_params(hrlb_mlp* m, const float* d_params);
int hrlb_mlp_get_params(hrlb_mlp* m, float* d_params);

/* Forward pass of rows input rows (d_x) into the raw outputs d_y[rows][8]. */
int hrlb_mlp_forward(hrlb_mlp* m, const float* d_x, int rows, float* d_y);

/* Forward pass written as a moment table d_table[rows][14] (fp64, the column order of
 * hrlb_moments) under the symmetries of plane Couette flow: u_x = u_z = 0,
 * P_xz = P_yz = 0, q_z = 0 and P_zz = 3 n T - P_xx - P_yy.  Feeds hrlb_seed_state. */
int hrlb_mlp_predict_table(hrlb_mlp* m, const float* d_x, int rows, double* d_table);

/* Loss and its gradient for rows rows, taken from the inputs d_x and targets d_t (raw
 * values) at the row indices d_idx[rows] (device; NULL = rows 0..rows-1).  d_grad
 * (device, flat layout) receives the gradient; d_loss (device, 1 float, may be NULL) the
 * loss.  The weights are not changed. */
int hrlb_mlp_gradient(hrlb_mlp* m, const float* d_x, const float* d_t, const int* d_idx, int rows, float* d_grad,
                      float* d_loss);

/* One AdamW step on the loss of the rows selected as in hrlb_mlp_gradient, with learning
 * rate lr > 0 and weight decay wd >= 0. */
int hrlb_mlp_train_step(hrlb_mlp* m, const float* d_x, const float* d_t, const int* d_idx, int rows, float lr,
                        float wd, float* d_loss);

void hrlb_mlp_free(hrlb_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* HRLB_MLP_H */
