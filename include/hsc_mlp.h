/* hsc_mlp.h: the surrogate network of the learned energy grid.
 *
 * A fully connected network in FP32, widths w[0] -> w[1] -> ... -> w[L-1], tanh on every
 * hidden layer and the identity on the output layer.  It maps (E, disorder sigma, Nx, Ny) to
 * (log DOS, log T) of a device; it is trained on the solver's own outputs and proposes where an
 * adaptive energy grid needs points.  Every call enqueues on the stream of the context;
 * arrays are device memory unless stated otherwise.
 *
 * Parameter layout (one flat float array, P values): for each layer l = 0 .. L-2 the weight
 * matrix W_l (row-major, w[l+1] rows by w[l] columns) followed by the bias b_l (w[l+1]).
 * Forward: h_0 = x, h_{l+1} = tanh(W_l h_l + b_l) for hidden layers, y = W h + b at the end.
 * Loss: mean squared error over all n * w[L-1] outputs, (1/(n w_out)) sum (y - t)^2.
 * Optimiser: Adam (Kingma and Ba 2015), bias-corrected first and second moments.
 *
 * Errors: HSC_E_ARG for null handles, non-positive sizes or widths outside [1, 1024];
 * HSC_E_OOM when workspace allocation fails; HSC_E_HIP for a failed launch.
 */
#ifndef HSC_MLP_H
#define HSC_MLP_H

#include <stdint.h>

#include "hsc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsc_mlp hsc_mlp;

typedef struct {
  float lr;       /* step size, e.g. 1e-3 */
  float beta1;    /* first-moment decay, e.g. 0.9 */
  float beta2;    /* second-moment decay, e.g. 0.999 */
  float eps;      /* denominator guard, e.g. 1e-8 */
  int32_t batch;  /* samples per step; batch >= n with order == NULL means full batch */
  int32_t steps;  /* Adam steps to take */
} hsc_train_opts;

/* Create a network with n_widths layer widths (n_widths >= 2).  Parameters are zero and the
 * Adam state is empty until hsc_mlp_set_params.  The network belongs to the context's device. */
hsc_status hsc_mlp_create(hsc_ctx* ctx, int32_t n_widths, const int32_t* widths /* host */, hsc_mlp** out);
hsc_status hsc_mlp_destroy(hsc_mlp* mlp);

/* Number of parameters P (host output). */
hsc_status hsc_mlp_n_params(const hsc_mlp* mlp, int64_t* out);

/* Copy P parameters in (device, float) and reset the Adam moments and step counter. */
hsc_status hsc_mlp_set_params(hsc_ctx* ctx, hsc_mlp* mlp, const float* params);
/* Copy the P parameters out (device, float). */
hsc_status hsc_mlp_get_params(hsc_ctx* ctx, const hsc_mlp* mlp, float* params);

/* y[n][w_out] = network(x[n][w_in]); row-major. */
hsc_status hsc_mlp_forward(hsc_ctx* ctx, hsc_mlp* mlp, int64_t n, const float* x, float* y);

/* Gradient of the mean squared error on (x, t) with respect to all P parameters, written to
 * grads (device, P floats, same layout as the parameters), and the loss to loss (device, 1). */
hsc_status hsc_mlp_grads(hsc_ctx* ctx, hsc_mlp* mlp, int64_t n, const float* x, const float* t, float* grads,
                         float* loss);

/* opts->steps Adam steps on (x, t).  Step s uses the samples order[s*batch .. s*batch+batch-1]
 * (device int32, values in [0, n)); with order == NULL every step uses all n samples.  The loss
 * of each step's batch, before its update, goes to loss_hist[s] (device, optional). */
hsc_status hsc_mlp_train(hsc_ctx* ctx, hsc_mlp* mlp, int64_t n, const float* x, const float* t,
                         const hsc_train_opts* opts, const int32_t* order, float* loss_hist);

#ifdef __cplusplus
}
#endif

#endif
