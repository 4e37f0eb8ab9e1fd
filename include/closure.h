/*
 * closure.h -- C ABI of the learned closure: a small convolutional network
 * that advances the filtered, projected velocity field u_M of the DPD
 * suspension (Sec. 5.4, Eqs. 5.8-5.10) by a fixed interval of DPD steps, with
 * its training (forward, backward, Adam) and rollout on the GPU.
 *
 * The network: L periodic 3 x 3 convolutions (cross-correlations with
 * wrap-around at the grid edges, the field being periodic like the box),
 * ReLU between them, width H, input channels c_in = (u_x, u_y, then c_in - 2
 * constant conditioning channels such as the friction and the propulsion of
 * the run), output 2 channels added to the input field:
 *     u(t + interval) = u(t) + net(u(t), conditions).
 * Weights are kept in FP32 (master copy, Adam moments) and enter every
 * convolution rounded to BF16; activations are rounded to BF16 where they enter
 * a convolution; every sum accumulates in FP32.  The forward and the
 * input-gradient convolutions are matrix-core products (BF16 in, FP32 out); the
 * weight gradients are FP32 sums over all pixels in a fixed order, so a
 * gradient is reproducible bit for bit.
 *
 * Conventions:
 *   - Fields are device FP32 arrays [B][M][M][2] (row j, column i, component),
 *     conditions device FP32 [B][c_in - 2]; all pointers device unless stated.
 *   - Parameters are one FP32 vector of dpd_nn_param_count values: for each
 *     layer l, its weights W_l[tap][c][o] (tap = 3 (dy + 1) + (dx + 1) for
 *     the input pixel at offset (dx, dy)), then its biases b_l[o].
 *   - The caller owns every buffer and the workspace; the library allocates no
 *     device memory.  Work is enqueued on the stream given to dpd_nn_create.
 *   - Return value: 0 or a negative DPD_E* code of dpd.h; dpd_nn_last_error
 *     gives the message.
 */
#ifndef DPD_CLOSURE_H
#define DPD_CLOSURE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dpd_nn_params {
    int32_t M;          /* grid side, multiple of 4, 4..256                     */
    int32_t c_in;       /* input channels, multiple of 4, 4..32 (2 are u)       */
    int32_t width;      /* hidden width H: 16 or 32                             */
    int32_t layers;     /* convolutions L, 1..8 (L = 1: a single 3 x 3 layer)   */
    int32_t max_batch;  /* largest batch B of a call, >= 1                      */
    int32_t reserved[3];
} dpd_nn_params;

typedef struct dpd_nn dpd_nn;

/* Number of FP32 parameters, and bytes of workspace, for p. */
int dpd_nn_param_count(const dpd_nn_params* p, int64_t* count);
int dpd_nn_workspace_bytes(const dpd_nn_params* p, size_t* bytes);

/* Carve the workspace (256-byte aligned, dpd_nn_workspace_bytes bytes) and
 * bind to `stream`.  Weights start at zero; set them with dpd_nn_set_weights.
 * Errors: DPD_EINVAL, DPD_EWORKSPACE. */
int dpd_nn_create(const dpd_nn_params* p, void* workspace, size_t bytes, void* stream,
                  dpd_nn** out);
void dpd_nn_destroy(dpd_nn* nn);
const char* dpd_nn_last_error(const dpd_nn* nn);

/* Set the FP32 parameters (and clear the Adam moments and step count), or read
 * them back. */
int dpd_nn_set_weights(dpd_nn* nn, const float* w);
int dpd_nn_get_weights(dpd_nn* nn, float* w);

/* pred = u + net(u, cond) for a batch of B fields. */
int dpd_nn_forward(dpd_nn* nn, const float* u, const float* cond, int32_t B, float* pred);

/* Loss = mean over B M M 2 values of (pred - target)^2, written to the
 * device double *loss (may be NULL), and its gradient with respect to the
 * parameters into grad (FP32, parameter layout). */
int dpd_nn_gradient(dpd_nn* nn, const float* u, const float* cond, const float* target,
                    int32_t B, float* grad, double* loss);

/* One Adam step (Kingma & Ba) on the master weights with gradient grad:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2, w -= lr mh / (sqrt(vh) + eps)
 * with the bias-corrected mh, vh of the step count t (incremented first). */
int dpd_nn_adam(dpd_nn* nn, const float* grad, float lr, float beta1, float beta2, float eps);

/* Gradient and Adam step in one call (the loss of the step in *loss). */
int dpd_nn_train_step(dpd_nn* nn, const float* u, const float* cond, const float* target,
                      int32_t B, float lr, float beta1, float beta2, float eps, double* loss);

/* Autonomous rollout of B fields (1 <= B <= max_batch) from u0 ([B][M][M][2])
 * under cond ([B][c_in - 2]): steps applications of the network, each
 * followed by noise.  White Gaussian numbers w (Philox4x32-10, counter
 * (b M^2 + grid point, component, step), key seed, Box-Muller) either enter as
 * noise_std[c] w (noise_filter NULL) or, with a filter h ([M][M] device,
 * M <= 64, B <= 65535, shared by the B fields), as noise_std[c] (h * w) with *
 * the periodic convolution (evaluated as IDFT(DFT(h) DFT(w)) with FP32 DFTs),
 * which gives the noise the spectrum |DFT(h)|^2 (a filter
 * h = IDFT(M sqrt(R)) gives normalised Fourier coefficients of power R(k) per
 * component).  noise_std: host, 2 values.  Every save_every-th set of fields
 * (k = save_every, 2 save_every, ...) is written to traj[k / save_every - 1]
 * ([B][M][M][2] each; traj holds steps / save_every of them).  The fields
 * stay in the workspace between the applications; u0 and cond are read once,
 * in stream order.  For c_in = 4, width 32, 2 to 4 layers and M in {32, 64}
 * a step is one kernel (the whole network on bands of rows in LDS, the noise
 * added in its last layer) and the noise of up to 8 steps is drawn ahead, in
 * the workspace's gradient buffers (filtered noise through two-stage
 * transforms); the network's part of every step is bitwise that of the
 * layer-by-layer kernels.  Errors: DPD_EINVAL, DPD_EHIP. */
int dpd_nn_rollout(dpd_nn* nn, const float* u0, const float* cond, int32_t B, int32_t steps,
                   const float* noise_std, const float* noise_filter, uint64_t seed,
                   int32_t save_every, float* traj);

/* Wait for the stream. */
int dpd_nn_sync(dpd_nn* nn);

/* ---- field statistics -------------------------------------------------------- */

/* Power spectrum of nfields fields u[f][M][M][2] (Sec. 5.4, Eqs. 5.11-5.12):
 * with the Fourier coefficients u^(k) = sum_{j,i} u[j][i] e^{-2 pi i (l j + k i)/M}
 * / M^2 of each component, power[l][k] = sum over the fields and the two
 * components of |u^(l, k)|^2 (device FP64, M x M; l the row wavenumber index,
 * k the column one, both 0..M-1).  The energy spectrum is half its shell sums,
 * and by Wiener-Khinchin its inverse transform is the fields' circular
 * autocorrelation.  work: device scratch of 4 nfields M^2 floats.  Enqueued on
 * `stream`.  Errors: DPD_EINVAL, DPD_EHIP. */
int dpd_field_power(const float* u, int32_t nfields, int32_t M, float* work, double* power,
                    void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DPD_CLOSURE_H */
