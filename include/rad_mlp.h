/*
 * rad_mlp.h -- C ABI of the BF16 MLP of the learned angular sampler (part of librad).
 *
 * The sampler (a form of the radiation-integral path grown beside the plain
 * FP64 kernel; it is not in the paper) predicts the log-intensity
 * log d2I/(d hw dOmega) over (hw, thx, thy) from trajectory features, and decides
 * where the angular grid is refined; the exact integrals of include/rad.h
 * (rad_batch on a coarse grid, rad_cells on the refined cells) stay the reference
 * for its error.  The network: inputs [n_feat trajectory features, n_point point
 * inputs] (n_feat + n_point <= 64) -> 256 -> 256 -> 256 -> 1, SiLU activations,
 * BF16 weights and activations, FP32 accumulation (the dense products run on
 * the MFMA units), mean-squared-error loss, Adam with FP32 master weights.
 *
 * Parameter vector (FP32, this order): W1 [256][n_feat + n_point] (rows are
 * outputs; the trajectory features first), b1 [256], W2 [256][256], b2 [256],
 * W3 [256][256], b3 [256], W4 [256], b4 [1].
 *
 * Conventions as in rad.h: DEVICE pointers are GPU memory on the current device,
 * HOST pointers CPU memory; `stream` is a hipStream_t; every call returns a
 * status and validates before it launches; compute calls use the caller's
 * workspace and allocate no device memory (rad_mlp_create allocates the
 * parameters, the Adam moments and the BF16 working copies).
 *
 * Batches: `traj[m]` (DEVICE int [batch]) is the trajectory of point m, an index
 * into `feat` (DEVICE float [n_traj][n_feat]); `x` (DEVICE float [batch][n_point])
 * the point inputs.  Internally a batch is padded to a multiple of 64 points.
 */
#ifndef RAD_MLP_H
#define RAD_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "rad.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rad_mlp rad_mlp;

/* Allocate a network and initialise it from `seed` (uniform +-sqrt(6/fan_in) for
 * the hidden layers, +-sqrt(6/fan_in)/4 for the output layer, zero biases).
 * RAD_EINVAL if n_feat < 0, n_point < 1 or n_feat + n_point > 64. */
rad_status rad_mlp_create(int n_feat, int n_point, uint64_t seed, void *stream, rad_mlp **out);
void rad_mlp_free(rad_mlp *mlp);
int64_t rad_mlp_param_count(const rad_mlp *mlp);

/* Copy the FP32 master parameters out / in (HOST float [param_count]); setting
 * them refreshes the BF16 working copies.  Both synchronise `stream`. */
rad_status rad_mlp_get_params(const rad_mlp *mlp, float *host, void *stream);
rad_status rad_mlp_set_params(rad_mlp *mlp, const float *host, void *stream);

/* Adam state for checkpoints: first and second moments (HOST float [param_count]
 * each, either may be NULL) and the step count. */
rad_status rad_mlp_get_adam(const rad_mlp *mlp, float *m1, float *m2, int64_t *step, void *stream);
rad_status rad_mlp_set_adam(rad_mlp *mlp, const float *m1, const float *m2, int64_t step, void *stream);

/* Workspace bytes for up to `batch` points and `n_traj` trajectories: of
 * rad_mlp_grad when `training` != 0, of rad_mlp_forward otherwise. */
size_t rad_mlp_workspace_bytes(const rad_mlp *mlp, int batch, int n_traj, int training);

/* Gradient of the mean squared error (1/B) sum_m (y_m - target_m)^2 with respect
 * to every parameter: grad (DEVICE float [param_count]); loss_sum (DEVICE float
 * [1]) receives sum_m (y_m - target_m)^2.  Deterministic (fixed-order sums). */
rad_status rad_mlp_grad(const rad_mlp *mlp, const float *feat, int n_traj, const int *traj, const float *x,
                        const float *target, int batch, float *grad, float *loss_sum, void *ws,
                        size_t ws_bytes, void *stream);

/* One Adam step on the master parameters with gradient `grad` (DEVICE), then the
 * BF16 copies are refreshed.  Increments the step count. */
rad_status rad_mlp_adam(rad_mlp *mlp, const float *grad, float lr, float beta1, float beta2, float eps,
                        void *stream);

/* Inference y (DEVICE float [batch]): the trajectory part of layer 1 is folded into
 * one bias per trajectory, so layer 1 costs n_point products per unit and point.
 * With n_point <= 8 one fused kernel runs the whole network for 32 points per wave
 * (activations stay in registers, W2 in LDS); otherwise layer by layer.  The values
 * of traj must lie in [0, n_traj). */
rad_status rad_mlp_forward(const rad_mlp *mlp, const float *feat, int n_traj, const int *traj, const float *x,
                           int batch, float *y, void *ws, size_t ws_bytes, void *stream);

/* Inference over every (trajectory, point) pair without per-point inputs: x (DEVICE
 * float [n_pts][n_point]) is one table of point inputs shared by all trajectories, y
 * (DEVICE float [n_traj][n_pts]) receives the output of trajectory t at point i in
 * y[t * n_pts + i].  Needs n_point <= 8 (the fused kernel; RAD_EUNSUPPORTED
 * otherwise); ws: DEVICE workspace of rad_mlp_grid_workspace_bytes(mlp, n_traj)
 * bytes (the folded biases). */
size_t rad_mlp_grid_workspace_bytes(const rad_mlp *mlp, int n_traj);
rad_status rad_mlp_forward_grid(const rad_mlp *mlp, const float *feat, int n_traj, const float *x, int64_t n_pts,
                                float *y, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAD_MLP_H */
