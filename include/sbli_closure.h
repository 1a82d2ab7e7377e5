/*
 * sbli_closure.h -- C ABI of the learned closure of libsbli.so: a small periodic
 * 3D convolutional network that corrects the residual of a coarse solver, its
 * training kernels (BF16 MFMA with FP32 accumulation on gfx950) and the box
 * filter that makes its training data from fine-grid solutions.
 *
 * This part is not in the paper, which names large-eddy-simulation models as
 * future work (Sec. "Introduction") on top of the same residual evaluation.
 * It is used for the "learned-closure" form: coarse state q_c (FP32, 5 planar
 * fields) -> network -> closure term C with the same shape, added to the
 * coarse residual inside each RK3 stage (sbli_closure_attach).
 *
 * Network: conv3d 5->32, GELU, conv3d 32->32, GELU, conv3d 32->5, every kernel
 * 3x3x3 with periodic wrap, biases, exact (erf) GELU.  Inputs are standardised
 * per channel with "input" statistics; outputs are standardised "output"
 * statistics (training targets are standardised the same way).  Parameters are
 * one flat FP32 vector, per layer W[out][in][3][3][3] (kernel index
 * (dz+1)*9 + (dy+1)*3 + (dx+1), cross-correlation) then b[out]: 36357 values.
 * The convolutions run on BF16 copies of weights and activations with FP32
 * accumulation; the FP32 master parameters are updated by Adam.
 *
 * Conventions as in sbli.h: int status, device pointers for arrays unless a
 * name says host, all work on the stream given at creation.  Planar state
 * arrays are [batch][5][n][n][n] FP32.
 */
#ifndef SBLI_CLOSURE_H
#define SBLI_CLOSURE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbli_net sbli_net;

/* Create a network for n^3 periodic grids (n a multiple of 32, <= 1024) with
 * workspaces for up to max_batch samples.  Parameters start at zero and the
 * statistics at mean 0 / std 1 with no guard limit. */
int sbli_net_create(int n, int max_batch, void* hip_stream, sbli_net** out);
int sbli_net_destroy(sbli_net* net);
const char* sbli_net_last_error(const sbli_net* net);
int sbli_net_num_params(const sbli_net* net);
int sbli_net_n(const sbli_net* net);

/* Host copies of the flat FP32 parameter vector.  set_params also resets the
 * Adam moments and step count. */
int sbli_net_set_params(sbli_net* net, const float* host_params);
int sbli_net_get_params(sbli_net* net, float* host_params);
/* Host copy of the gradients left by the last sbli_net_gradients / train_step. */
int sbli_net_get_grads(sbli_net* net, float* host_grads);

/* Statistics, 35 floats: [0..4] input means, [5..9] input standard deviations,
 * [10..14] output means, [15..19] output standard deviations, [20..24] per-field
 * guard limits on |C| (see sbli_net_guard), [25..29] / [30..34] largest |value|
 * per field of the input / output samples.  sbli_net_channel_stats computes the
 * population mean, standard deviation (FP64 sums) and largest magnitude per
 * field of `count` planar samples on the device into the input (which = 0) or
 * output (which = 1) slots. */
int sbli_net_set_stats(sbli_net* net, const float* host_stats);
int sbli_net_get_stats(sbli_net* net, float* host_stats);
int sbli_net_channel_stats(sbli_net* net, const float* data, int count, int which);

/* out = destandardised network output for `batch` planar samples q. */
int sbli_net_forward(sbli_net* net, const float* q, int batch, float* out);
/* Forward, mean-squared error against the standardised `target` (planar, raw
 * units), backward; gradients stay on the device (sbli_net_get_grads).
 * *loss (host, may be NULL) receives the loss; then the stream is synchronised. */
int sbli_net_gradients(sbli_net* net, const float* q, const float* target, int batch, double* loss);
/* sbli_net_gradients followed by one Adam step (beta = 0.9, 0.999, eps 1e-8,
 * bias-corrected) with learning rate lr. */
int sbli_net_train_step(sbli_net* net, const float* q, const float* target, int batch, float lr, double* loss);
/* flag[0] = 1 if every value of the planar closure term c (one sample) is finite
 * and within the guard limit of its field, else 0; counters[0] / counters[1]
 * are incremented for accepted / rejected evaluations. */
int sbli_net_guard(sbli_net* net, const float* c, int* flag, unsigned* counters);

/* Box filter of `nfields` planar fields of an nf^3 periodic grid (dtype SBLI_F64
 * or SBLI_F32) onto the (nf/ratio)^3 grid: separable centred trapezoid of width
 * ratio*h (weights 1/(2 ratio) at +-ratio/2, 1/ratio between), coarse point i on
 * fine point ratio*i, FP32 output.  subtract = 0: coarse = F(fine); otherwise
 * coarse = F(fine) - coarse (in place; e.g. a closure target F R_f - R_c). */
int sbli_box_filter(const void* fine, int dtype, int nf, int nfields, int ratio, float* coarse, int subtract,
                    void* hip_stream);

/* Attach a trained network to a solver context (FP32, cubic grid of the net's
 * n): every RK3 stage of sbli_rk3_step then evaluates C = net(q_stage) and, if
 * sbli_net_guard accepts it, uses R(q) + C instead of R(q) (otherwise the plain
 * residual: the fallback).  net = NULL detaches.  The network must outlive the
 * attachment.  sbli_closure_counts returns the accepted / rejected counts. */
int sbli_closure_attach(struct sbli_ctx* ctx, sbli_net* net);
int sbli_closure_counts(struct sbli_ctx* ctx, unsigned counts[2]);

#ifdef __cplusplus
}
#endif

#endif /* SBLI_CLOSURE_H */
