/* msx_flow.h -- learned importance sampler of the phase-space library: a
 * rational-quadratic spline coupling flow (Durkan et al. 2019) stacked in
 * front of the VEGAS-mapped channel of a msx context.
 *
 * The paper's adaptive-sampling section (2.3) names normalizing flows built
 * from rational-quadratic spline transformations as its neural importance
 * sampler and defers their details; the single-bin case of the spline is the
 * RQF of the FastRambo mapping (section 2.2.9).  This interface fixes:
 *
 *  - The flow maps u in (0,1)^d to y in (0,1)^d through `layers` coupling
 *    layers.  Layer l transforms one half of the coordinates given the other
 *    half: l mod 4 = 0 the first d/2, 1 the last d/2, 2 the even ones, 3 the
 *    odd ones.  Each transformed coordinate goes through a monotone spline of
 *    `bins` rational-quadratic bins on [0,1].  Its 3 bins + 1 parameters come
 *    from an MLP  d/2 -> hidden -> hidden -> hidden -> (d/2)(3 bins + 1) with
 *    ReLU after each hidden layer.  Output column j (3 bins + 1) + q is
 *    parameter q of transformed coordinate j: q < bins are the widths,
 *    q < 2 bins the heights, the rest the bins + 1 knot slopes.
 *  - Widths / heights are 1e-3 + (1 - bins 1e-3) softmax(theta).  Slopes are
 *    1e-3 + softplus(theta + log(e^(1 - 1e-3) - 1)).  All parameters zero give
 *    the identity map.
 *  - Parameters are FP32, flat.  Per layer, in order: W1 [hidden][d/2], b1,
 *    W2 [hidden][hidden], b2, W3 [hidden][hidden], b3,
 *    W4 [(d/2)(3 bins + 1)][hidden], b4.  Layers follow one another.
 *  - MSX_FLOW_BF16: the MLP runs on the matrix cores with BF16 inputs,
 *    weights and hidden activations and FP32 accumulation; biases are FP32.
 *    MSX_FLOW_FP32: FP32 operands throughout.  The spline, the loss and Adam
 *    are FP32 in both modes.
 *  - Event arrays are device pointers owned by the caller, SoA: u, y [d][n]
 *    float; per-event scalars [n].  Calls enqueue on `stream` (a hipStream_t,
 *    NULL = default stream) and return without waiting.
 *  - Errors: MSX_ERR_ARG for bad arguments (no launch); device failures
 *    as in msx.h.  The text is returned by msx_flow_last_error.
 */
#ifndef MSX_FLOW_H
#define MSX_FLOW_H

#include <stdint.h>

#include "msx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msx_flow msx_flow;

enum { MSX_FLOW_BF16 = 0, MSX_FLOW_FP32 = 1 };

/* Text of the last error on this flow (or of the last failed create when
 * flow is NULL). */
const char* msx_flow_last_error(const msx_flow* flow);

/* New flow on device `device`, parameters all zero (identity), Adam state
 * zero.  dims even, 2..64; layers 1..64; bins 1..32; hidden 1..1024. */
msx_status msx_flow_create(int32_t dims, int32_t layers, int32_t bins, int32_t hidden, int32_t mlp_type,
                           int32_t device, msx_flow** out);
msx_status msx_flow_destroy(msx_flow* flow);

/* Random dimensions d of the flow. */
msx_status msx_flow_dims(const msx_flow* flow, int32_t* dims);

/* The flow's trainable state as one host blob: shape, FP32 master
 * parameters, Adam's moments m and v and its step count (checkpoint /
 * resume).  get: buf NULL sets *size to the bytes needed (16 + 32 + 12 P);
 * set: restores a blob of a flow of the same shape and type (else
 * MSX_ERR_STATE; non-finite values are refused).  Both synchronise. */
msx_status msx_flow_get_state(msx_flow* flow, void* buf, size_t* size);
msx_status msx_flow_set_state(msx_flow* flow, const void* buf, size_t size);

/* Number of FP32 parameters. */
msx_status msx_flow_param_count(const msx_flow* flow, int64_t* n);

/* Copy parameters in from / out to host memory (n must equal the count).
 * set_params also clears the Adam moments and step count.  Both synchronise
 * the device. */
msx_status msx_flow_set_params(msx_flow* flow, const float* host_params, int64_t n);
msx_status msx_flow_get_params(msx_flow* flow, float* host_params, int64_t n);

/* y = flow(u) and logdet = log |det dy/du| for n events. */
msx_status msx_flow_forward(msx_flow* flow, int64_t n, const float* u, float* y, float* logdet, void* stream);

/* u = flow^-1(y) and logq = log |det du/dy| (the log density of y). */
msx_status msx_flow_inverse(msx_flow* flow, int64_t n, const float* y, float* u, float* logq, void* stream);

/* Variance loss of a batch drawn from the flow,
 *   L = (1/n) sum_i wfj_i^2 exp(-logq(y_i) - logq_old_i),
 * with wfj_i = f J of the event (its weight without the flow density) and
 * logq_old_i the flow's log density when the event was drawn.  Writes the
 * loss to loss[0] (device double) and dL/dparams to grad [P] (device).
 * Gradients run through the inverse pass. */
msx_status msx_flow_gradient(msx_flow* flow, int64_t n, const float* y, const double* wfj, const float* logq_old,
                             float* grad, double* loss, void* stream);

/* One Adam step (beta 0.9, 0.999, eps 1e-8, learning rate lr) on the
 * gradient of log L (the direction of msx_flow_gradient's, divided by L: free
 * of the integrand's units, so eps does not interact with the weight scale).
 * loss[0] (device, optional) receives L. */
msx_status msx_flow_train_step(msx_flow* flow, int64_t n, const float* y, const double* wfj, const float* logq_old,
                               float lr, double* loss, void* stream);

/* Attach a trained flow to channel `channel` of ctx for MSX_SAMPLE_USE_FLOW
 * sample calls (flow NULL detaches).  The flow must have the channel's
 * dimension and outlive its attachment; the context does not own it.  With
 * n_check > 0 the library decides whether to use it -- the fallback to plain
 * VEGAS: it draws n_check events through the channel's VEGAS grid alone and
 * n_check through the flow (msx_flow_sample), and enables the flow only if
 * its relative weight variance var(w)/mean(w)^2 is the lower one (at equal
 * event count the flow then reaches a smaller integral error).  n_check = 0
 * enables it unconditionally.  *enabled (optional) gets the decision,
 * rel_var[2] (optional) the two relative variances (VEGAS, flow; NaN without
 * a check).  Synchronises. */
msx_status msx_attach_flow(msx_ctx* ctx, int32_t channel, msx_flow* flow, int64_t n_check, uint64_t seed,
                           int32_t* enabled, double* rel_var);

/* Production path of the learned sampler for one channel of `ctx` (whose
 * dims must equal the flow's): 24-bit Philox uniforms u (key (seed,
 * stream_id), counter (counter_offset + i, k / 4, 0, 0)) -> y = flow(u) ->
 * msx_map (VEGAS grid, mapping chain, integrand, channel weight) -> w.
 * Outputs: y [d][n] float, logq [n] float (log density of y), p, x1x2 as in
 * msx_map, wfj [n] (f J without the flow density) and w [n] = wfj / q(y). */
msx_status msx_flow_sample(msx_flow* flow, msx_ctx* ctx, int32_t channel, int64_t n, uint64_t seed,
                           uint64_t stream_id, uint64_t counter_offset, float* y, float* logq, double* p,
                           double* x1x2, double* wfj, double* w, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MSX_FLOW_H */
