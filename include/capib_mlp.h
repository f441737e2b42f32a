/* capib_mlp.h — the load/hazard surrogate of the capillary-adhesion solver.
 *
 * A multilayer perceptron that maps 37 features of an adhered particle's
 * situation (cell to particle distance r, cell membrane stretch dp, particle
 * aspect ratio, log10 Ca, cell type, and a 32-sample history of the wall
 * shear stress under the particle) to 3 outputs (hydrodynamic drag and lift
 * on the particle, Eqs. 14-15 summed over its elements, and the bond
 * rupture hazard, the mean Bell rupture probability of its engaged bonds,
 * Sec. 2.5).  Four hidden layers of width 256 with GELU, a linear output.
 * It screens a parameter sweep before the full LBM-IB solver is run; the
 * solver produces its training data and measures its error.
 *
 * Arithmetic: bfloat16 inputs, weights and activations, FP32 accumulation
 * on the matrix cores; FP32 master weights updated by Adam.  Rounding to
 * bfloat16 (nearest, ties to even) happens at: the input, the weights, the
 * hidden activations, the output gradient and every back-propagated
 * pre-activation gradient.
 *
 * Ownership: as for capib.h — the caller owns the device workspace (bound
 * once); the library keeps host metadata only.  Feature, target and output
 * arrays named "device" are device pointers in the caller's memory; all work
 * is enqueued on the stream given at creation.
 *
 * Parameter vector (FP32, CAPIB_MLP_PARAMS floats): W0 [256][37], b0 [256],
 * W1 [256][256], b1, W2 [256][256], b2, W3 [256][256], b3, W4 [3][256],
 * b4 [3]; each W row-major [out][in].
 */
#ifndef CAPIB_MLP_H
#define CAPIB_MLP_H

#include "capib.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { CAPIB_MLP_IN = 37, CAPIB_MLP_HIDDEN = 256, CAPIB_MLP_OUT = 3, CAPIB_MLP_PARAMS = 207875 };

typedef struct capib_mlp capib_mlp;

/* Creates a surrogate for batches of up to max_batch samples (>= 1).
 * hip_stream: hipStream_t or NULL.                                         */
capib_status capib_mlp_create(int32_t max_batch, void *hip_stream, capib_mlp **out);

/* Device workspace bytes; bind a 256-byte-aligned buffer of that size once
 * (weights are then zero; set them with capib_mlp_set_params).             */
size_t capib_mlp_workspace_bytes(const capib_mlp *m);
capib_status capib_mlp_bind_workspace(capib_mlp *m, void *device_ptr, size_t bytes);

/* Copies the FP32 parameter vector in (host array, CAPIB_MLP_PARAMS floats;
 * resets the Adam state) or out.  Non-finite values are refused.  Syncs.   */
capib_status capib_mlp_set_params(capib_mlp *m, const float *params);
capib_status capib_mlp_get_params(capib_mlp *m, float *params);

/* Inference: y [n][3] = net(x [n][37]), FP32 device arrays, 1 <= n <=
 * max_batch.  Enqueued.                                                    */
capib_status capib_mlp_forward(capib_mlp *m, const float *x_device, int32_t n, float *y_device);

/* Loss and gradients for a batch: mean over the batch and the 3 outputs of
 * (y - t)^2 with t [n][3] (device).  The gradients stay in the workspace
 * for capib_mlp_adam_step; if grads (host, CAPIB_MLP_PARAMS floats, same
 * layout as the parameters) is not NULL they are copied out, and if loss
 * (host) is not NULL the loss is returned; either copy syncs.              */
capib_status capib_mlp_loss_grad(capib_mlp *m, const float *x_device, const float *t_device, int32_t n,
                                 double *loss, float *grads);

/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8) of every parameter
 * with the gradients of the last capib_mlp_loss_grad.  Enqueued.          */
capib_status capib_mlp_adam_step(capib_mlp *m, float lr);

const char *capib_mlp_last_error(const capib_mlp *m);
void capib_mlp_destroy(capib_mlp *m);

#ifdef __cplusplus
}
#endif
#endif
