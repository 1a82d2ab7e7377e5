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
/* Release a network: waits for its stream, frees every buffer even when a HIP
 * call fails, and returns the first failure (SBLI_ERR_HIP, message from
 * sbli_net_last_error(NULL)).  NULL is a no-op. */
int sbli_net_destroy(sbli_net* net);
const char* sbli_net_last_error(const sbli_net* net);
int sbli_net_num_params(const sbli_net* net);
int sbli_net_n(const sbli_net* net);
/* The hipStream_t given at creation (every call of the network enqueues there). */
void* sbli_net_stream(const sbli_net* net);

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

/* out = destandardised network output for `batch` planar samples q.  In the
 * conservative mode (sbli_net_set_conservative) each output field of each
 * sample then has its box mean removed (FP64 sums in a fixed order), so that
 * the closure term adds nothing to the totals of mass, momentum and energy,
 * as the exact term F R_f - R_c(F q_f) does (both residuals are in the
 * conservative form of Sec. "3D Taylor-Green vortex"; the filter keeps totals). */
int sbli_net_forward(sbli_net* net, const float* q, int batch, float* out);
/* Conservative mode of sbli_net_forward (and so of the closure term a solver
 * adds through sbli_closure_attach): on = 1 removes the box means, 0 (the
 * default) leaves the output as computed.  SBLI_ERR_ARG for other values. */
int sbli_net_set_conservative(sbli_net* net, int on);
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

/*
 * ---- The network's kernels, one call each ----
 * These are the kernels sbli_net_* runs, exported with explicit device
 * pointers, shapes and stream so that each one can be driven (and checked) on
 * its own.  They run asynchronously on `hip_stream` and touch only the buffers
 * passed in.
 *
 * Activation layout: BF16, channel-last [batch][n^3][cpad] (point index
 * (z*n + y)*n + x, x fastest), cpad = sbli_conv3d_cpad(channels): 8 for up to 8
 * channels, 32 for 9..32.  Padding channels must hold finite values (zeros
 * recommended); they meet zero weights.  n is a multiple of 32 in [32, 1024]
 * and batch * n^3 <= 2^31.  Convolution: out[p][o] = b[o] + sum_{c, tap}
 * W[o][c][tap] in[p + off(tap)][c], 3x3x3 taps with periodic wrap, tap =
 * (dz+1)*9 + (dy+1)*3 + (dx+1) (cross-correlation, as in every network layer
 * above), FP32 accumulation of exact BF16 products.
 */

/* cpad for `channels` (1..32), or SBLI_ERR_ARG. */
int sbli_conv3d_cpad(int channels);
/* Width of a packed weight row for `channels` input channels (forward) or
 * output channels (backward-data): round_up(27 * cpad(channels), 16). */
int sbli_conv3d_packed_width(int channels);

/* Pack FP32 master weights W[cout][cin][27] (device) into the BF16 operand
 * layouts of the two convolution kernels (round to nearest even):
 *   Wf[32][Kf], Kf = packed_width(cin):  Wf[o][tap*cpad(cin) + c]     = W[o][c][tap]
 *   Wb[32][Kb], Kb = packed_width(cout): Wb[c][tap'*cpad(cout) + o]   = W[o][c][26 - tap']
 * (the mirrored tap makes backward-data a convolution of the same kind); every
 * other entry is 0.  Either output may be NULL.  1 <= cin, cout <= 32. */
int sbli_conv3d_pack(const float* W, int cin, int cout, void* Wf, void* Wb, void* hip_stream);

#define SBLI_ACT_NONE 0
#define SBLI_ACT_GELU 1
/* Forward convolution on MFMA (v_mfma_f32_32x32x16_bf16, LDS-staged input box)
 * of x [batch][n^3][cpad(cin)] with packed Wf and FP32 bias b[cout]:
 *   act = SBLI_ACT_GELU (cout = 32): pre[batch][n^3][32] (FP32) = conv + b and
 *     h[batch][n^3][32] (BF16) = bf16(gelu(pre)), exact-erf GELU in FP32;
 *   act = SBLI_ACT_NONE: pre[batch][n^3][cpad(cout)] (FP32), channels < cout
 *     written (the padding channels are left as they are); h unused (NULL).
 * x must not overlap the outputs. */
int sbli_conv3d_fwd(const void* x, int cin, const void* Wf, const float* b, int cout, int n, int batch, int act,
                    float* pre, void* h, void* hip_stream);

/* Backward-data convolution (the data gradient of a layer with cin = 32 input
 * channels): g[p][c] = sum_{o, tap} W[o][c][tap] dy[p - off(tap)][o], with dy
 * [batch][n^3][cpad(cout)] BF16 and packed Wb.
 *   pre != NULL: dx[batch][n^3][32] BF16 = bf16(g * gelu'(pre)), pre the FP32
 *     pre-activation [batch][n^3][32] of the layer below (GELU' fused into the
 *     epilogue: this is how the network runs);
 *   pre == NULL: dx[batch][n^3][32] FP32 = g.
 * dy must not overlap dx. */
int sbli_conv3d_bwd_data(const void* dy, int cout, const void* Wb, int n, int batch, const float* pre, void* dx,
                         void* hip_stream);

/* Element-wise GELU backward: dx[i] = bf16(g[i] * gelu'(pre[i])) for `count`
 * FP32 values g and pre (gelu'(v) = Phi(v) + v phi(v), FP32).  With g from
 * sbli_conv3d_bwd_data(pre = NULL) this gives bitwise the fused epilogue. */
int sbli_gelu_bwd(const float* g, const float* pre, long long count, void* dx, void* hip_stream);

/* Device workspace (bytes) that sbli_conv3d_bwd_weight needs for `cin` input
 * channels (partial sums of a fixed number of workgroups), or < 0 on error. */
long long sbli_conv3d_bwd_weight_work_bytes(int cin);
/* Weight and bias gradients of a convolution: dW[o][c][tap] = sum_{b, p}
 * dy[b][p][o] x[b][p + off(tap)][c] and db[o] = sum_{b, p} dy[b][p][o] (FP32,
 * o < cout, c < cin; dW in the master layout, db may be NULL), x [batch][n^3]
 * [cpad(cin)] and dy [batch][n^3][cpad(cout)] BF16.  Every sum runs in a fixed
 * order (deterministic).  `work` is device memory of at least
 * sbli_conv3d_bwd_weight_work_bytes(cin) bytes. */
int sbli_conv3d_bwd_weight(const void* x, int cin, const void* dy, int cout, int n, int batch, float* dW, float* db,
                           void* work, long long work_bytes, void* hip_stream);

/* Device workspace (bytes) that sbli_mse_grad needs, or < 0 on error. */
long long sbli_mse_grad_work_bytes(int n, int batch);
/* Mean-squared error of the network output y [batch][n^3][ystride] (FP32,
 * channels 0..4 used; ystride must be 8, the layout sbli_conv3d_fwd writes for
 * 5 output channels) against the standardised planar target
 * t [batch][5][n^3] (FP32, standardised here with mean_std[0..4] / [5..9],
 * device): loss[0] (device double) = sum (y - t_std)^2 / (5 batch n^3), and its
 * gradient dy[batch][n^3][8] (BF16, channels 5..7 zero) = bf16(2 (y - t_std) /
 * (5 batch n^3)).  `work` holds at least sbli_mse_grad_work_bytes bytes. */
int sbli_mse_grad(const float* y, int ystride, const float* t, const float* mean_std, int n, int batch, void* dy,
                  double* loss, void* work, long long work_bytes, void* hip_stream);

/* sbli_mse_grad for callers that cannot allocate (code under HIP graph capture,
 * tight training loops, harnesses that forbid hipMalloc): the same kernels and
 * results, with no `work` argument.  The loss partials go to a static device
 * array of the library (512 KiB per GPU, held until the process ends), so
 * batch * n^3 <= 2^24 (SBLI_ERR_ARG beyond).  The call allocates nothing.  Calls
 * on one GPU share that array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be ordered by the caller. */
int sbli_mse_grad_noalloc(const float* y, int ystride, const float* t, const float* mean_std, int n, int batch,
                          void* dy, double* loss, void* hip_stream);

/* One Adam step (Kingma & Ba, bias-corrected, beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8) on `count` FP32 values in place:
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * t >= 1 is the step number (1 for the first step); lr > 0. */
int sbli_adam_step(float* p, const float* g, float* m, float* v, int count, float lr, int t, void* hip_stream);

/* Attach a trained network to a solver context (FP32, cubic grid of the net's
 * n, and created on the solver's stream: SBLI_ERR_ARG otherwise, since the
 * stage kernel reads the closure term the network writes): every RK3 stage of sbli_rk3_step then evaluates C = net(q_stage) and, if
 * sbli_net_guard accepts it, uses R(q) + C instead of R(q) (otherwise the plain
 * residual: the fallback).  net = NULL detaches.  The network must outlive the
 * attachment.  sbli_closure_counts returns the accepted / rejected counts. */
int sbli_closure_attach(struct sbli_ctx* ctx, sbli_net* net);
int sbli_closure_counts(struct sbli_ctx* ctx, unsigned counts[2]);

#ifdef __cplusplus
}
#endif

#endif /* SBLI_CLOSURE_H */
