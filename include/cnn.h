/*
 * libhmc -- the small 3-D CNN of the learned warm start and mass.
 *
 * Not part of the paper's method: the paper notes that the mass matrix affects
 * only efficiency, not validity (text after eq. Mass_matrix), and that a
 * start closer to the posterior shortens burn-in (Sec. "Testing burn-in and
 * statistical efficiency").  This network supplies both: from three input
 * fields (normalised data, angular mask, radial selection) it predicts the
 * posterior mean mu and log-variance s of the density per voxel.
 *
 * Architecture: four 3x3x3 convolutions (zero padding) 3 -> 16 -> 16 -> 16 -> 2,
 * GELU after the first three.  Weights are bfloat16 MFMA operands with float32
 * accumulation; float32 master weights and Adam state live on the device.
 * Loss: mean_i 1/2 [(x_i - mu_i)^2 exp(-s_i) + s_i] against a training draw x.
 *
 * Parameter vector (host float32, cnn_param_count() values): for each layer
 * l = 0..3 with (C_in, C_out) = (3,16), (16,16), (16,16), (16,2): weights
 * W[27][C_in][C_out] then bias[C_out]; tap t = 9 (dx+1) + 3 (dy+1) + (dz+1)
 * and z[v, o] = b[o] + sum_t sum_c a[v + (dx, dy, dz)_t, c] W[t, c, o].
 *
 * Buffers: inputs, targets and outputs are caller-owned device float32 arrays
 * of N^3 voxels (row-major [x][y][z]); activations and gradients live in
 * device memory owned by the context (allocated on the first call for a given
 * N, freed by cnn_destroy).  All work runs on `stream`; calls returning host
 * values synchronise it.  Errors as in hmc.h (HMC_EINVAL: N not a multiple of 4
 * or < 4, null pointers).
 */
#ifndef LIBHMC_CNN_H
#define LIBHMC_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "hmc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cnn_ctx cnn_ctx;

/* Number of float32 parameters (weights and biases of the four layers). */
size_t cnn_param_count(void);

/* New network on `stream` with the given initial parameters (host float32,
 * cnn_param_count() values). */
hmc_status cnn_create(const float* params, void* stream, cnn_ctx** out);

/* Copy the float32 master parameters to the host. */
hmc_status cnn_get_params(cnn_ctx* ctx, float* params);

/* Forward pass.  in3: device [3][N^3] (channel 0 normalised data, 1 mask,
 * 2 selection); mu, logvar: device [N^3] outputs (either may be NULL). */
hmc_status cnn_forward(cnn_ctx* ctx, int32_t n, const float* in3, float* mu, float* logvar);

/* Network inputs from the survey: out3 (device [3][N^3]) receives
 * beta * beta_scale (the data combination beta_i = sum_l b_l (N^l_i - Nbar_l
 * R^l_i) of the force, normalised by the caller, e.g. 1 / sum_l b_l^2 Nbar_l),
 * the angular mask and the radial selection (device [N^3] each). */
hmc_status cnn_features(cnn_ctx* ctx, int32_t n, const float* beta, float beta_scale,
                        const float* mask, const float* sel, float* out3);

/* Loss and gradients without updating (host outputs; grad may be NULL). */
hmc_status cnn_gradient(cnn_ctx* ctx, int32_t n, const float* in3, const float* target,
                        float* grad, double* loss);

/* One Adam step (beta1 0.9, beta2 0.999, epsilon 1e-8, bias-corrected) with
 * learning rate lr on the loss against target (device [N^3]); loss: host. */
hmc_status cnn_train_step(cnn_ctx* ctx, int32_t n, const float* in3, const float* target,
                          float lr, double* loss);

/* The stored state of layer `layer` (0..3) from the last cnn_gradient or
 * cnn_train_step, as float32 device arrays [N^3][C_out] (C_out = 16, or 2 for
 * layer 3), any of which may be NULL: z the pre-activations (float32 sums
 * plus bias), a the bfloat16 activations GELU(z) that feed the next layer (NULL
 * for layer 3, which has none), dz the bfloat16 gradient of the loss with
 * respect to z.  They let a test check one layer at a time from the layer's own
 * inputs (the rounding points of the network are its bf16 weights, activations
 * and output gradients).  HMC_EINVAL if no gradient was evaluated since the
 * context was created, its grid size changed or cnn_forward ran. */
hmc_status cnn_layer_state(cnn_ctx* ctx, int32_t layer, float* z, float* a, float* dz);

const char* cnn_last_error(const cnn_ctx* ctx);
void cnn_destroy(cnn_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
