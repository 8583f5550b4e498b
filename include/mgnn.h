/*
 * mgnn.h -- C ABI of the learned warm start for the multigrid Poisson solve.
 *
 * The paper contains no learned component.  This network predicts an initial
 * potential phi0 for mg_solve (include/mg.h) from the density; plain multigrid
 * from a zero guess is its fallback and the measure of its error.
 *
 * Network: five 3x3x3 convolutions with circular (periodic) padding on an
 * n^3 grid, widths 1 -> 24 -> 24 -> 24 -> 24 -> 1, bias on every layer,
 * GELU u/2 (1 + erf(u/sqrt 2)) after the first four (erf by Abramowitz &
 * Stegun 7.1.26: within 6e-7 in FP32, far below the BF16 resolution of the
 * activations).  Weights and stored
 * activations are bfloat16 (round to nearest even), products accumulate in
 * FP32 (the 24 -> 24 layers on the matrix cores), master weights and Adam
 * state are FP32.  Input x = f / rms(f) with f = four_pi_G (rho - rho_mean)
 * (equivalently f h^2 / s with s = std(f h^2)); output phi0 = s y.
 *
 * Dense fields of the *_raw calls are [n^3] arrays indexed (x n + y) n + z
 * (z fastest).  Fields of mgnn_forward / mgnn_train_step use the oct-major
 * layout of a full periodic level (see mg.h).  Parameters travel as one flat
 * FP32 vector: for each layer l = 0..4, W_l[o][c][t] then b_l[o], with tap
 * t = 9 (dx+1) + 3 (dy+1) + (dz+1) for the input read at offset (dx,dy,dz).
 *
 * Device pointers are owned by the caller; the handle owns its parameters,
 * optimiser state and workspaces (grown on demand to the largest n used).
 * Work is enqueued on `stream`; calls that return host values synchronise.
 * A handle is not thread-safe.  Errors are reported as in mg.h.
 */
#ifndef MGNN_H_
#define MGNN_H_

#include <stdint.h>

#include "mg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgnn_s* mgnn_t;

/* channels must be 24 and layers 5; weights get a seeded He-normal
 * initialisation (std sqrt(2 / (27 c_in))), biases 0. */
mg_status_t mgnn_create(int32_t channels, int32_t layers, uint64_t seed, mgnn_t* out);
void mgnn_destroy(mgnn_t net);

/* Number of FP32 parameters (48049 for 24 channels, 5 layers). */
int64_t mgnn_num_params(mgnn_t net);
mg_status_t mgnn_get_weights(mgnn_t net, float* h_buf, int64_t n);
mg_status_t mgnn_set_weights(mgnn_t net, const float* h_buf, int64_t n);
/* Accumulated gradients (same layout as the weights). */
mg_status_t mgnn_get_grads(mgnn_t net, float* h_buf, int64_t n);
mg_status_t mgnn_zero_grad(mgnn_t net, void* stream);

/* Forward pass on a normalised input: d_x [n^3] f32 (rounded to bf16 on entry)
 * -> d_y [n^3] f32.  Keeps the activations for mgnn_backward_raw.
 * n: power of two, 8 <= n <= 1024. */
mg_status_t mgnn_forward_raw(mgnn_t net, int32_t n, const float* d_x, float* d_y, void* stream);

/* Backward pass of the last mgnn_forward_raw / mgnn_train_step forward:
 * d_dy = dL/dy [n^3] f32; adds dL/dW, dL/db to the gradient buffer; writes
 * dL/dx to d_dx [n^3] f32 when d_dx is not NULL. */
mg_status_t mgnn_backward_raw(mgnn_t net, int32_t n, const float* d_dy, float* d_dx, void* stream);

/* Backward pass of the field form: d_dloss_dphi = dL/dphi0 [(n/2)^3][8] f32,
 * oct-major, the gradient of a loss with respect to the phi0 of the last
 * mgnn_forward on this handle (which must have been at this n, with no raw
 * pass or training step since).  Adds dL/dW, dL/db to the gradient buffer,
 * with the scale s = h^2 rms(f) of that forward held fixed (dL/dy = s dL/dphi0).
 * mgnn_forward keeps only the network input, so this call first recomputes
 * the activations with the current weights.  MG_ERR_ARG without a matching
 * forward. */
mg_status_t mgnn_backward(mgnn_t net, int32_t n, const float* d_dloss_dphi, void* stream);

/* One Adam step on all parameters with the accumulated gradients (bias-
 * corrected; the step counter is kept by the handle). */
mg_status_t mgnn_adam_step(mgnn_t net, float lr, float b1, float b2, float eps, void* stream);

/* Warm start: phi0 = s * net(f / rms(f)), f = four_pi_G (rho - rho_mean),
 * s = h^2 rms(f), h = 1/n.  d_rho, d_phi0: [(n/2)^3][8] f64 oct-major.
 * rho_mean: NAN = FP64 mean of d_rho. */
mg_status_t mgnn_forward(mgnn_t net, int32_t n, const double* d_rho, double rho_mean, double four_pi_G,
                         double* d_phi0, void* stream);

/* One training step on one field: forward, loss, backward, Adam (lr, 0.9,
 * 0.999, 1e-8).  With t = phi_target / s,
 * loss = sum((y - t)^2) / sum(t^2) + res_weight * mean(R^2),
 * R = x - Lap(y), Lap the periodic 7-point Laplacian in lattice units:
 * R is the residual f - L_h phi0 of the warm start divided by rms(f), so
 * mean(R^2) is its squared relative residual.  d_phi_target: oct-major f64 (a
 * multigrid solution).  *h_loss receives the loss (synchronises). */
mg_status_t mgnn_train_step(mgnn_t net, int32_t n, const double* d_rho, double rho_mean, double four_pi_G,
                            const double* d_phi_target, float lr, float res_weight, double* h_loss, void* stream);

/* Warm-started solve on a periodic level L (n = L's base_n): phi0 from
 * mgnn_forward; if ||f - L phi0|| / ||f|| is not finite or not below 1 the
 * guess is replaced by zero (*used_fallback = 1 and info->used_fallback = 1;
 * used_fallback may be NULL).  Then mg_solve from that guess.  info->ms
 * covers the whole call (network + check + solve).  Returns mg_solve's
 * status. */
mg_status_t mgnn_solve_warm(mgnn_t net, mg_level_t L, const double* d_rho, double rho_mean, double four_pi_G,
                            double* d_phi, double tol, int32_t max_cycles, mg_solve_info_t* info,
                            int32_t* used_fallback);

#ifdef __cplusplus
}
#endif

#endif /* MGNN_H_ */
