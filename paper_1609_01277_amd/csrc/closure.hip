// libsbli: host side of the learned closure (include/sbli_closure.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>

#include "../../include/sbli.h"
#include "../../include/sbli_closure.h"
#include "closure_kernels.h"

using namespace sbli;

namespace {

constexpr int kCh[4] = {5, 32, 32, 5};      // channels of the network
constexpr int kCpad[4] = {8, 32, 32, 8};    // padded channel strides of the activations

int round_up(int v, int m) { return (v + m - 1) / m * m; }

constexpr int kWgradWg = 512;   // workgroups of the weight-gradient kernel (fixed, so the sum order is fixed)

struct Layer {
    int cin, cout, cpad, opad;   // real and padded input / output channels
    int Kf, Kb, Kpad32;          // packed forward / backward-data widths, weight-gradient width
    size_t w_off, b_off;         // offsets of W [cout][cin][27] and b [cout] in the flat vector
    __bf16* Wf = nullptr;        // [32][Kf]
    __bf16* Wb = nullptr;        // [32][Kb]
};

}  // namespace

struct sbli_net {
    int n = 0, max_batch = 0;
    int64_t P = 0;
    hipStream_t stream = nullptr;
    Layer L[kNetLayers];
    int nparams = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    int adam_t = 0;
    float* stats = nullptr;          // [0..9] input mean/std, [10..19] output mean/std, [20..24] guard
                                     // limits, [25..29] input max |x|, [30..34] output max |x|
    __bf16 *x = nullptr, *h1 = nullptr, *h2 = nullptr, *dy = nullptr, *d2 = nullptr, *d1 = nullptr;
    float *pre1 = nullptr, *pre2 = nullptr, *y = nullptr;
    float* wpart = nullptr;          // weight-gradient partials
    float* bpart = nullptr;          // bias-gradient partials [kBiasWg][32]
    int wgrad_wg = kWgradWg;
    double* loss_part = nullptr;
    double* loss = nullptr;
    int conservative = 0;            // remove each output field's box mean in sbli_net_forward
    double* mean_part = nullptr;     // box-mean partial sums [max_batch * 5][chunks]
    float* mean_val = nullptr;       // box means [max_batch * 5]
    std::string err;
};

static std::string g_net_err;

static int nfail(sbli_net* net, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (net) net->err = buf;
    else g_net_err = buf;
    return code;
}

#define NHIP_TRY(net, call)                                                                          \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return nfail(net, SBLI_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

extern "C" const char* sbli_net_last_error(const sbli_net* net) { return net ? net->err.c_str() : g_net_err.c_str(); }

extern "C" int sbli_net_destroy(sbli_net* net) {
    if (!net) return SBLI_OK;
    // everything is released whatever fails; the first failure is reported
    hipError_t first = hipStreamSynchronize(net->stream);
    auto release = [&](void* p) {
        const hipError_t e = hipFree(p);
        if (first == hipSuccess) first = e;
    };
    for (int l = 0; l < kNetLayers; ++l) {
        release(net->L[l].Wf);
        release(net->L[l].Wb);
    }
    void* ptrs[] = {net->params, net->grads, net->adam_m, net->adam_v, net->stats, net->x, net->h1, net->h2,
                    net->dy, net->d2, net->d1, net->pre1, net->pre2, net->y, net->wpart, net->bpart, net->loss_part,
                    net->loss, net->mean_part, net->mean_val};
    for (void* p : ptrs) release(p);
    delete net;
    if (first != hipSuccess) return nfail(nullptr, SBLI_ERR_HIP, "sbli_net_destroy: %s", hipGetErrorString(first));
    return SBLI_OK;
}

extern "C" int sbli_net_create(int n, int max_batch, void* hip_stream, sbli_net** out) {
    if (!out) return nfail(nullptr, SBLI_ERR_ARG, "sbli_net_create: out is NULL");
    *out = nullptr;
    if (n < 32 || n % 32 != 0 || n > 1024)
        return nfail(nullptr, SBLI_ERR_ARG, "sbli_net_create: n must be a multiple of 32 in [32, 1024] (got %d)", n);
    if (max_batch < 1 || (int64_t)max_batch * n * n * n > (int64_t)1 << 31)
        return nfail(nullptr, SBLI_ERR_ARG, "sbli_net_create: max_batch out of range");
    sbli_net* net = new (std::nothrow) sbli_net();
    if (!net) return nfail(nullptr, SBLI_ERR_ALLOC, "sbli_net_create: out of host memory");
    net->n = n;
    net->max_batch = max_batch;
    net->P = (int64_t)n * n * n;
    net->stream = (hipStream_t)hip_stream;
    size_t off = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        Layer& L = net->L[l];
        L.cin = kCh[l];
        L.cout = kCh[l + 1];
        L.cpad = kCpad[l];
        L.opad = kCpad[l + 1];
        L.Kf = round_up(27 * L.cpad, 16);
        L.Kb = round_up(27 * L.opad, 16);
        L.Kpad32 = round_up(27 * L.cpad, 32);
        L.w_off = off;
        off += (size_t)L.cout * L.cin * 27;
        L.b_off = off;
        off += L.cout;
    }
    net->nparams = (int)off;
    const int64_t NP = (int64_t)max_batch * net->P;
    hipError_t e = hipSuccess;
    auto alloc = [&](void** p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
        if (e == hipSuccess) e = hipMemsetAsync(*p, 0, bytes, net->stream);
    };
    for (int l = 0; l < kNetLayers; ++l) {
        alloc((void**)&net->L[l].Wf, sizeof(__bf16) * 32 * net->L[l].Kf);
        alloc((void**)&net->L[l].Wb, sizeof(__bf16) * 32 * net->L[l].Kb);
    }
    alloc((void**)&net->params, sizeof(float) * net->nparams);
    alloc((void**)&net->grads, sizeof(float) * net->nparams);
    alloc((void**)&net->adam_m, sizeof(float) * net->nparams);
    alloc((void**)&net->adam_v, sizeof(float) * net->nparams);
    alloc((void**)&net->stats, sizeof(float) * 40);
    alloc((void**)&net->x, sizeof(__bf16) * NP * 8);
    alloc((void**)&net->h1, sizeof(__bf16) * NP * 32);
    alloc((void**)&net->h2, sizeof(__bf16) * NP * 32);
    alloc((void**)&net->dy, sizeof(__bf16) * NP * 8);
    alloc((void**)&net->d2, sizeof(__bf16) * NP * 32);
    alloc((void**)&net->d1, sizeof(__bf16) * NP * 32);
    alloc((void**)&net->pre1, sizeof(float) * NP * 32);
    alloc((void**)&net->pre2, sizeof(float) * NP * 32);
    alloc((void**)&net->y, sizeof(float) * NP * 8);
    alloc((void**)&net->wpart, sizeof(float) * (size_t)net->wgrad_wg * 32 * 27 * 32);
    alloc((void**)&net->bpart, sizeof(float) * (size_t)kBiasWg * 32);
    alloc((void**)&net->loss_part, sizeof(double) * nblk(NP));
    alloc((void**)&net->loss, sizeof(double));
    alloc((void**)&net->mean_part, sizeof(double) * (size_t)max_batch * 5 * nblk(net->P, kBoxMeanChunk));
    alloc((void**)&net->mean_val, sizeof(float) * (size_t)max_batch * 5);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) {
        nfail(nullptr, e == hipErrorOutOfMemory ? SBLI_ERR_ALLOC : SBLI_ERR_HIP, "sbli_net_create: %s",
              hipGetErrorString(e));
        sbli_net_destroy(net);
        return e == hipErrorOutOfMemory ? SBLI_ERR_ALLOC : SBLI_ERR_HIP;
    }
    // identity standardisation until set: mean 0, std 1, no guard limit
    float st[40] = {0};
    for (int c = 0; c < 5; ++c) {
        st[5 + c] = 1.0f;
        st[15 + c] = 1.0f;
        st[20 + c] = INFINITY;
    }
    e = hipMemcpyAsync(net->stats, st, sizeof(st), hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    if (e != hipSuccess) {
        nfail(nullptr, SBLI_ERR_HIP, "sbli_net_create: %s", hipGetErrorString(e));
        sbli_net_destroy(net);
        return SBLI_ERR_HIP;
    }
    *out = net;
    return SBLI_OK;
}

extern "C" int sbli_net_num_params(const sbli_net* net) {
    if (!net) return nfail(nullptr, SBLI_ERR_ARG, "sbli_net_num_params: net is NULL");
    return net->nparams;
}

static int pack_all(sbli_net* net) {
    for (int l = 0; l < kNetLayers; ++l) {
        const Layer& L = net->L[l];
        const int tot = 32 * (L.Kf > L.Kb ? L.Kf : L.Kb);
        pack_weights_kernel<<<nblk(tot), 256, 0, net->stream>>>(net->params + L.w_off, L.cin, L.cout, L.cpad, L.opad,
                                                                L.Kf, L.Kb, L.Wf, L.Wb);
    }
    NHIP_TRY(net, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_net_set_params(sbli_net* net, const float* host_params) {
    if (!net || !host_params) return nfail(net, SBLI_ERR_ARG, "sbli_net_set_params: NULL argument");
    NHIP_TRY(net, hipMemcpyAsync(net->params, host_params, sizeof(float) * net->nparams, hipMemcpyHostToDevice,
                                 net->stream));
    NHIP_TRY(net, hipMemsetAsync(net->adam_m, 0, sizeof(float) * net->nparams, net->stream));
    NHIP_TRY(net, hipMemsetAsync(net->adam_v, 0, sizeof(float) * net->nparams, net->stream));
    net->adam_t = 0;
    int rc = pack_all(net);
    if (rc != SBLI_OK) return rc;
    NHIP_TRY(net, hipStreamSynchronize(net->stream));
    return SBLI_OK;
}

extern "C" int sbli_net_get_params(sbli_net* net, float* host_params) {
    if (!net || !host_params) return nfail(net, SBLI_ERR_ARG, "sbli_net_get_params: NULL argument");
    NHIP_TRY(net, hipMemcpyAsync(host_params, net->params, sizeof(float) * net->nparams, hipMemcpyDeviceToHost,
                                 net->stream));
    NHIP_TRY(net, hipStreamSynchronize(net->stream));
    return SBLI_OK;
}

extern "C" int sbli_net_get_grads(sbli_net* net, float* host_grads) {
    if (!net || !host_grads) return nfail(net, SBLI_ERR_ARG, "sbli_net_get_grads: NULL argument");
    NHIP_TRY(net, hipMemcpyAsync(host_grads, net->grads, sizeof(float) * net->nparams, hipMemcpyDeviceToHost,
                                 net->stream));
    NHIP_TRY(net, hipStreamSynchronize(net->stream));
    return SBLI_OK;
}

extern "C" int sbli_net_channel_stats(sbli_net* net, const float* data, int count, int which) {
    if (!net || !data) return nfail(net, SBLI_ERR_ARG, "sbli_net_channel_stats: NULL argument");
    if (count < 1 || (which != 0 && which != 1))
        return nfail(net, SBLI_ERR_ARG, "sbli_net_channel_stats: count >= 1 and which in {0, 1} required");
    channel_stats_kernel<<<5, 256, 0, net->stream>>>(data, count, net->P, net->stats + 10 * which,
                                                    net->stats + 25 + 5 * which);
    NHIP_TRY(net, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_net_set_stats(sbli_net* net, const float* host_stats) {
    if (!net || !host_stats) return nfail(net, SBLI_ERR_ARG, "sbli_net_set_stats: NULL argument");
    for (int c = 0; c < 5; ++c)
        if (!(host_stats[5 + c] > 0) || !(host_stats[15 + c] > 0))
            return nfail(net, SBLI_ERR_ARG, "sbli_net_set_stats: standard deviations must be > 0");
    NHIP_TRY(net, hipMemcpyAsync(net->stats, host_stats, sizeof(float) * 35, hipMemcpyHostToDevice, net->stream));
    NHIP_TRY(net, hipStreamSynchronize(net->stream));
    return SBLI_OK;
}

extern "C" int sbli_net_get_stats(sbli_net* net, float* host_stats) {
    if (!net || !host_stats) return nfail(net, SBLI_ERR_ARG, "sbli_net_get_stats: NULL argument");
    NHIP_TRY(net, hipMemcpyAsync(host_stats, net->stats, sizeof(float) * 35, hipMemcpyDeviceToHost, net->stream));
    NHIP_TRY(net, hipStreamSynchronize(net->stream));
    return SBLI_OK;
}

// One convolution (implicit GEMM on MFMA, input staged in LDS): `in` has cpad
// channels per point (8 or 32), epilogue EPI (see closure_kernels.h).  The
// network and the per-kernel exports launch it through here.
template <int EPI>
static void conv_launch(hipStream_t stream, int n, const __bf16* in, int cpad, const __bf16* W, int Kpad,
                        const float* bias, int batch, float* fout, __bf16* bout, const float* pre_in, int ocount,
                        int ostride) {
    const unsigned g = (unsigned)((int64_t)batch * n * (n / kConvTy) * (n / kConvTx));
    if (cpad == 32)
        conv_mfma_lds_kernel<EPI, 32><<<g, 256, 0, stream>>>(in, W, Kpad, bias, n, fout, bout, pre_in, ocount,
                                                              ostride);
    else
        conv_mfma_lds_kernel<EPI, 8><<<g, 256, 0, stream>>>(in, W, Kpad, bias, n, fout, bout, pre_in, ocount,
                                                             ostride);
}

template <int EPI>
static void conv(sbli_net* net, const __bf16* in, int cpad, const __bf16* W, int Kpad, const float* bias, int batch,
                 float* fout, __bf16* bout, const float* pre_in, int ocount, int ostride) {
    conv_launch<EPI>(net->stream, net->n, in, cpad, W, Kpad, bias, batch, fout, bout, pre_in, ocount, ostride);
}

// Weight and bias gradients of one layer: per-workgroup partials, then fixed-order
// reductions into dW (master layout) and db.
static void wgrad_launch(hipStream_t stream, int n, int batch, const __bf16* in, int cpad, int cin, const __bf16* dout,
                         int opad, int cout, int nwg, float* wpart, float* bpart, float* dW, float* db) {
    const int Kpad32 = round_up(27 * cpad, 32);
    const int64_t blocks = (int64_t)batch * n * n * (n / 32);
    conv_wgrad_kernel<<<nwg, 256, 0, stream>>>(in, cpad, dout, opad, n, blocks, Kpad32, wpart);
    wgrad_reduce_kernel<<<nblk(cout * Kpad32), 256, 0, stream>>>(wpart, nwg, Kpad32, cpad, cin, cout, dW);
    if (db) {
        bias_grad_kernel<<<kBiasWg, 256, 0, stream>>>(dout, opad, (int64_t)batch * n * n * n, bpart);
        bias_grad_final_kernel<<<1, 256, 0, stream>>>(bpart, kBiasWg, cout, db);
    }
}

// Forward pass of `batch` samples: x -> h1 -> h2 -> y (all in the net's buffers).
static int forward_core(sbli_net* net, const float* q, int batch) {
    const int64_t NP = (int64_t)batch * net->P;
    standardize_kernel<<<nblk(NP), 256, 0, net->stream>>>(q, net->P, batch, net->stats, net->x);
    const Layer* L = net->L;
    conv<kEpiGelu>(net, net->x, L[0].cpad, L[0].Wf, L[0].Kf, net->params + L[0].b_off, batch, net->pre1, net->h1,
                   nullptr, 32, 32);
    conv<kEpiGelu>(net, net->h1, L[1].cpad, L[1].Wf, L[1].Kf, net->params + L[1].b_off, batch, net->pre2, net->h2,
                   nullptr, 32, 32);
    conv<kEpiLinear>(net, net->h2, L[2].cpad, L[2].Wf, L[2].Kf, net->params + L[2].b_off, batch, net->y, nullptr,
                     nullptr, L[2].cout, 8);
    NHIP_TRY(net, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_net_forward(sbli_net* net, const float* q, int batch, float* out) {
    if (!net || !q || !out) return nfail(net, SBLI_ERR_ARG, "sbli_net_forward: NULL argument");
    if (batch < 1 || batch > net->max_batch)
        return nfail(net, SBLI_ERR_ARG, "sbli_net_forward: batch must be in [1, %d]", net->max_batch);
    int rc = forward_core(net, q, batch);
    if (rc != SBLI_OK) return rc;
    const int64_t NP = (int64_t)batch * net->P;
    destandardize_kernel<<<nblk(NP), 256, 0, net->stream>>>(net->y, net->P, batch, net->stats + 10, out);
    if (net->conservative) {
        const int nchunks = (int)nblk(net->P, kBoxMeanChunk), nbf = 5 * batch;
        box_mean_partial_kernel<<<(unsigned)nchunks * (unsigned)nbf, 256, 0, net->stream>>>(out, net->P, nchunks,
                                                                                             net->mean_part);
        box_mean_final_kernel<<<nblk(nbf, 64), 64, 0, net->stream>>>(net->mean_part, nchunks, nbf, net->P,
                                                                      net->mean_val);
        box_mean_subtract_kernel<<<nblk((int64_t)nbf * net->P), 256, 0, net->stream>>>(out, net->P, nbf, net->mean_val);
    }
    NHIP_TRY(net, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_net_set_conservative(sbli_net* net, int on) {
    if (!net) return nfail(nullptr, SBLI_ERR_ARG, "sbli_net_set_conservative: net is NULL");
    if (on != 0 && on != 1) return nfail(net, SBLI_ERR_ARG, "sbli_net_set_conservative: on must be 0 or 1");
    net->conservative = on;
    return SBLI_OK;
}

static int wgrad(sbli_net* net, int l, const __bf16* in, const __bf16* dout, int batch) {
    const Layer& L = net->L[l];
    wgrad_launch(net->stream, net->n, batch, in, L.cpad, L.cin, dout, L.opad, L.cout, net->wgrad_wg, net->wpart,
                 net->bpart, net->grads + L.w_off, net->grads + L.b_off);
    NHIP_TRY(net, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_net_gradients(sbli_net* net, const float* q, const float* target, int batch, double* loss) {
    if (!net || !q || !target) return nfail(net, SBLI_ERR_ARG, "sbli_net_gradients: NULL argument");
    if (batch < 1 || batch > net->max_batch)
        return nfail(net, SBLI_ERR_ARG, "sbli_net_gradients: batch must be in [1, %d]", net->max_batch);
    int rc = forward_core(net, q, batch);
    if (rc != SBLI_OK) return rc;
    const int64_t NP = (int64_t)batch * net->P;
    const Layer* L = net->L;
    const unsigned g = nblk(NP);
    mse_grad_kernel<<<g, 256, 0, net->stream>>>(net->y, target, net->P, batch, net->stats + 10, net->dy, net->loss_part);
    sum_doubles_kernel<<<1, 256, 0, net->stream>>>(net->loss_part, (int)g, 1.0 / (5.0 * (double)NP), net->loss);
    // layer 3
    if ((rc = wgrad(net, 2, net->h2, net->dy, batch)) != SBLI_OK) return rc;
    conv<kEpiDGelu>(net, net->dy, L[2].opad, L[2].Wb, L[2].Kb, nullptr, batch, nullptr, net->d2, net->pre2, 32, 32);
    // layer 2
    if ((rc = wgrad(net, 1, net->h1, net->d2, batch)) != SBLI_OK) return rc;
    conv<kEpiDGelu>(net, net->d2, L[1].opad, L[1].Wb, L[1].Kb, nullptr, batch, nullptr, net->d1, net->pre1, 32, 32);
    // layer 1
    if ((rc = wgrad(net, 0, net->x, net->d1, batch)) != SBLI_OK) return rc;
    NHIP_TRY(net, hipGetLastError());
    if (loss) {
        NHIP_TRY(net, hipMemcpyAsync(loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, net->stream));
        NHIP_TRY(net, hipStreamSynchronize(net->stream));
    }
    return SBLI_OK;
}

extern "C" int sbli_net_train_step(sbli_net* net, const float* q, const float* target, int batch, float lr,
                                   double* loss) {
    if (!net) return nfail(nullptr, SBLI_ERR_ARG, "sbli_net_train_step: net is NULL");
    if (!(lr > 0) || !std::isfinite(lr)) return nfail(net, SBLI_ERR_ARG, "sbli_net_train_step: lr must be > 0");
    int rc = sbli_net_gradients(net, q, target, batch, nullptr);
    if (rc != SBLI_OK) return rc;
    net->adam_t += 1;
    adam_kernel<<<nblk(net->nparams), 256, 0, net->stream>>>(net->params, net->grads, net->adam_m, net->adam_v,
                                                             net->nparams, lr, 0.9f, 0.999f, 1e-8f, net->adam_t);
    NHIP_TRY(net, hipGetLastError());
    rc = pack_all(net);
    if (rc != SBLI_OK) return rc;
    if (loss) {
        NHIP_TRY(net, hipMemcpyAsync(loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, net->stream));
        NHIP_TRY(net, hipStreamSynchronize(net->stream));
    }
    return SBLI_OK;
}

extern "C" int sbli_net_guard(sbli_net* net, const float* c, int* flag, unsigned* counters) {
    if (!net || !c || !flag || !counters) return nfail(net, SBLI_ERR_ARG, "sbli_net_guard: NULL argument");
    closure_guard_kernel<<<1, 1024, 0, net->stream>>>(c, net->P, net->stats + 20, flag, counters);
    NHIP_TRY(net, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_net_n(const sbli_net* net) { return net ? net->n : SBLI_ERR_ARG; }

extern "C" void* sbli_net_stream(const sbli_net* net) { return net ? (void*)net->stream : nullptr; }

extern "C" int sbli_box_filter(const void* fine, int dtype, int nf, int nfields, int ratio, float* coarse,
                               int subtract, void* hip_stream) {
    if (!fine || !coarse) return nfail(nullptr, SBLI_ERR_ARG, "sbli_box_filter: NULL pointer");
    if (ratio < 2 || ratio % 2 || nf < 2 * ratio || nf % ratio || nfields < 1)
        return nfail(nullptr, SBLI_ERR_ARG, "sbli_box_filter: need an even ratio >= 2 dividing nf >= 2 ratio");
    if (dtype != SBLI_F64 && dtype != SBLI_F32) return nfail(nullptr, SBLI_ERR_ARG, "sbli_box_filter: bad dtype");
    const int nc = nf / ratio;
    const int64_t total = (int64_t)nc * nc * nc * nfields;
    hipStream_t s = (hipStream_t)hip_stream;
    if (dtype == SBLI_F64)
        box_filter_kernel<double><<<nblk(total), 256, 0, s>>>((const double*)fine, nf, nfields, ratio, coarse,
                                                              subtract);
    else
        box_filter_kernel<float><<<nblk(total), 256, 0, s>>>((const float*)fine, nf, nfields, ratio, coarse,
                                                             subtract);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(nullptr, SBLI_ERR_HIP, "sbli_box_filter: %s", hipGetErrorString(e));
    return SBLI_OK;
}

// ---------------------------------------------------------------------------
// The network's kernels as separate entry points (explicit pointers, shapes and
// stream).  Each validates its shapes on the host and launches exactly the
// kernels the network runs.

static int conv_cpad(int c) { return c >= 1 && c <= 8 ? 8 : (c >= 9 && c <= 32 ? 32 : -1); }

static int check_grid(const char* fn, int n, int batch) {
    if (n < 32 || n % 32 != 0 || n > 1024)
        return nfail(nullptr, SBLI_ERR_ARG, "%s: n must be a multiple of 32 in [32, 1024] (got %d)", fn, n);
    if (batch < 1 || (int64_t)batch * n * n * n > (int64_t)1 << 31)
        return nfail(nullptr, SBLI_ERR_ARG, "%s: batch must be >= 1 with batch * n^3 <= 2^31", fn);
    return SBLI_OK;
}

static int launch_status(const char* fn) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(nullptr, SBLI_ERR_HIP, "%s: %s", fn, hipGetErrorString(e));
    return SBLI_OK;
}

extern "C" int sbli_conv3d_cpad(int channels) {
    const int c = conv_cpad(channels);
    return c > 0 ? c : nfail(nullptr, SBLI_ERR_ARG, "sbli_conv3d_cpad: channels must be in [1, 32]");
}

extern "C" int sbli_conv3d_packed_width(int channels) {
    const int c = conv_cpad(channels);
    if (c < 0) return nfail(nullptr, SBLI_ERR_ARG, "sbli_conv3d_packed_width: channels must be in [1, 32]");
    return round_up(27 * c, 16);
}

extern "C" int sbli_conv3d_pack(const float* W, int cin, int cout, void* Wf, void* Wb, void* hip_stream) {
    if (!W || (!Wf && !Wb)) return nfail(nullptr, SBLI_ERR_ARG, "sbli_conv3d_pack: NULL argument");
    const int cpad = conv_cpad(cin), opad = conv_cpad(cout);
    if (cpad < 0 || opad < 0) return nfail(nullptr, SBLI_ERR_ARG, "sbli_conv3d_pack: cin, cout must be in [1, 32]");
    const int Kf = round_up(27 * cpad, 16), Kb = round_up(27 * opad, 16);
    pack_weights_kernel<<<nblk(32 * (Kf > Kb ? Kf : Kb)), 256, 0, (hipStream_t)hip_stream>>>(
        W, cin, cout, cpad, opad, Kf, Kb, (__bf16*)Wf, (__bf16*)Wb);
    return launch_status("sbli_conv3d_pack");
}

extern "C" int sbli_conv3d_fwd(const void* x, int cin, const void* Wf, const float* b, int cout, int n, int batch,
                               int act, float* pre, void* h, void* hip_stream) {
    const char* fn = "sbli_conv3d_fwd";
    if (!x || !Wf || !b || !pre) return nfail(nullptr, SBLI_ERR_ARG, "%s: NULL argument", fn);
    int rc = check_grid(fn, n, batch);
    if (rc != SBLI_OK) return rc;
    const int cpad = conv_cpad(cin), opad = conv_cpad(cout);
    if (cpad < 0 || opad < 0) return nfail(nullptr, SBLI_ERR_ARG, "%s: cin, cout must be in [1, 32]", fn);
    const int Kf = round_up(27 * cpad, 16);
    hipStream_t s = (hipStream_t)hip_stream;
    if (act == SBLI_ACT_GELU) {
        if (cout != 32 || !h) return nfail(nullptr, SBLI_ERR_ARG, "%s: GELU layers need cout = 32 and h", fn);
        conv_launch<kEpiGelu>(s, n, (const __bf16*)x, cpad, (const __bf16*)Wf, Kf, b, batch, pre, (__bf16*)h,
                              nullptr, 32, 32);
    } else if (act == SBLI_ACT_NONE) {
        conv_launch<kEpiLinear>(s, n, (const __bf16*)x, cpad, (const __bf16*)Wf, Kf, b, batch, pre, nullptr,
                                nullptr, cout, opad);
    } else {
        return nfail(nullptr, SBLI_ERR_ARG, "%s: act must be SBLI_ACT_NONE or SBLI_ACT_GELU", fn);
    }
    return launch_status(fn);
}

extern "C" int sbli_conv3d_bwd_data(const void* dy, int cout, const void* Wb, int n, int batch, const float* pre,
                                    void* dx, void* hip_stream) {
    const char* fn = "sbli_conv3d_bwd_data";
    if (!dy || !Wb || !dx) return nfail(nullptr, SBLI_ERR_ARG, "%s: NULL argument", fn);
    int rc = check_grid(fn, n, batch);
    if (rc != SBLI_OK) return rc;
    const int opad = conv_cpad(cout);
    if (opad < 0) return nfail(nullptr, SBLI_ERR_ARG, "%s: cout must be in [1, 32]", fn);
    const int Kb = round_up(27 * opad, 16);
    hipStream_t s = (hipStream_t)hip_stream;
    if (pre)
        conv_launch<kEpiDGelu>(s, n, (const __bf16*)dy, opad, (const __bf16*)Wb, Kb, nullptr, batch, nullptr,
                               (__bf16*)dx, pre, 32, 32);
    else
        conv_launch<kEpiData>(s, n, (const __bf16*)dy, opad, (const __bf16*)Wb, Kb, nullptr, batch, (float*)dx,
                              nullptr, nullptr, 32, 32);
    return launch_status(fn);
}

extern "C" int sbli_gelu_bwd(const float* g, const float* pre, long long count, void* dx, void* hip_stream) {
    if (!g || !pre || !dx) return nfail(nullptr, SBLI_ERR_ARG, "sbli_gelu_bwd: NULL argument");
    if (count < 0) return nfail(nullptr, SBLI_ERR_ARG, "sbli_gelu_bwd: count < 0");
    if (count == 0) return SBLI_OK;
    gelu_bwd_kernel<<<nblk(count), 256, 0, (hipStream_t)hip_stream>>>(g, pre, count, (__bf16*)dx);
    return launch_status("sbli_gelu_bwd");
}

extern "C" long long sbli_conv3d_bwd_weight_work_bytes(int cin) {
    const int cpad = conv_cpad(cin);
    if (cpad < 0) return nfail(nullptr, SBLI_ERR_ARG, "sbli_conv3d_bwd_weight_work_bytes: cin must be in [1, 32]");
    return (long long)sizeof(float) * ((long long)kWgradWg * 32 * round_up(27 * cpad, 32) + (long long)kBiasWg * 32);
}

extern "C" int sbli_conv3d_bwd_weight(const void* x, int cin, const void* dy, int cout, int n, int batch, float* dW,
                                      float* db, void* work, long long work_bytes, void* hip_stream) {
    const char* fn = "sbli_conv3d_bwd_weight";
    if (!x || !dy || !dW || !work) return nfail(nullptr, SBLI_ERR_ARG, "%s: NULL argument", fn);
    int rc = check_grid(fn, n, batch);
    if (rc != SBLI_OK) return rc;
    const int cpad = conv_cpad(cin), opad = conv_cpad(cout);
    if (cpad < 0 || opad < 0) return nfail(nullptr, SBLI_ERR_ARG, "%s: cin, cout must be in [1, 32]", fn);
    const long long need = sbli_conv3d_bwd_weight_work_bytes(cin);
    if (work_bytes < need) return nfail(nullptr, SBLI_ERR_ARG, "%s: work holds %lld bytes, %lld needed", fn, work_bytes, need);
    float* wpart = (float*)work;
    float* bpart = wpart + (size_t)kWgradWg * 32 * round_up(27 * cpad, 32);
    wgrad_launch((hipStream_t)hip_stream, n, batch, (const __bf16*)x, cpad, cin, (const __bf16*)dy, opad, cout,
                 kWgradWg, wpart, bpart, dW, db);
    return launch_status(fn);
}

// MSE partials per block into `part` (one double per 256 points), then their sum.
static void mse_launch(hipStream_t s, const float* y, const float* t, const float* mean_std, int n, int batch,
                       void* dy, double* loss, double* part) {
    const int64_t NP = (int64_t)batch * n * n * n;
    const unsigned g = nblk(NP);
    mse_grad_kernel<<<g, 256, 0, s>>>(y, t, (int64_t)n * n * n, batch, mean_std, (__bf16*)dy, part);
    sum_doubles_kernel<<<1, 256, 0, s>>>(part, (int)g, 1.0 / (5.0 * (double)NP), loss);
}

extern "C" long long sbli_mse_grad_work_bytes(int n, int batch) {
    if (check_grid("sbli_mse_grad_work_bytes", n, batch) != SBLI_OK) return SBLI_ERR_ARG;
    return (long long)sizeof(double) * nblk((int64_t)batch * n * n * n);
}

extern "C" int sbli_mse_grad(const float* y, int ystride, const float* t, const float* mean_std, int n, int batch,
                             void* dy, double* loss, void* work, long long work_bytes, void* hip_stream) {
    const char* fn = "sbli_mse_grad";
    if (!y || !t || !mean_std || !dy || !loss || !work) return nfail(nullptr, SBLI_ERR_ARG, "%s: NULL argument", fn);
    int rc = check_grid(fn, n, batch);
    if (rc != SBLI_OK) return rc;
    if (ystride != 8) return nfail(nullptr, SBLI_ERR_ARG, "%s: ystride must be 8 (the padded output layout)", fn);
    const int64_t NP = (int64_t)batch * n * n * n;
    if (work_bytes < (long long)sizeof(double) * nblk(NP))
        return nfail(nullptr, SBLI_ERR_ARG, "%s: work is too small", fn);
    mse_launch((hipStream_t)hip_stream, y, t, mean_std, n, batch, dy, loss, (double*)work);
    return launch_status(fn);
}

// ---------------------------------------------------------------------------
// sbli_mse_grad without a workspace argument: the per-block loss partials go to a
// file-scope device array instead.  Each GPU holds its own copy of the array; its
// address on a device is looked up once (hipGetSymbolAddress, with that device
// current) and kept per device.  Nothing in it needs to start at zero: every
// block writes its own partial before the final sum reads it.  Calls that overlap
// on one GPU share the array and race.

constexpr int kMseScratchDoubles = 1 << 16;    // 512 KiB: batch * n^3 <= 2^24 points
static __device__ __align__(256) double scratch[kMseScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
static int scratch_on_current_device(const char* fn, double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return nfail(nullptr, SBLI_ERR_HIP, "%s: hipGetDevice: %s", fn, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return nfail(nullptr, SBLI_ERR_UNSUPPORTED, "%s: device %d", fn, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return nfail(nullptr, SBLI_ERR_HIP, "%s: hipGetSymbolAddress(scratch): %s", fn, hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return SBLI_OK;
}

extern "C" int sbli_mse_grad_noalloc(const float* y, int ystride, const float* t, const float* mean_std, int n,
                                     int batch, void* dy, double* loss, void* hip_stream) {
    const char* fn = "sbli_mse_grad_noalloc";
    if (!y || !t || !mean_std || !dy || !loss) return nfail(nullptr, SBLI_ERR_ARG, "%s: NULL argument", fn);
    int rc = check_grid(fn, n, batch);
    if (rc != SBLI_OK) return rc;
    if (ystride != 8) return nfail(nullptr, SBLI_ERR_ARG, "%s: ystride must be 8 (the padded output layout)", fn);
    const int64_t NP = (int64_t)batch * n * n * n;
    if (nblk(NP) > (unsigned)kMseScratchDoubles)
        return nfail(nullptr, SBLI_ERR_ARG, "%s: batch * n^3 = %lld exceeds the maximum %lld of the static scratch",
                     fn, (long long)NP, (long long)kMseScratchDoubles * 256);
    double* part = nullptr;
    rc = scratch_on_current_device(fn, &part);
    if (rc != SBLI_OK) return rc;
    mse_launch((hipStream_t)hip_stream, y, t, mean_std, n, batch, dy, loss, part);
    return launch_status(fn);
}

extern "C" int sbli_adam_step(float* p, const float* g, float* m, float* v, int count, float lr, int t,
                              void* hip_stream) {
    if (!p || !g || !m || !v) return nfail(nullptr, SBLI_ERR_ARG, "sbli_adam_step: NULL argument");
    if (count < 0 || t < 1 || !(lr > 0) || !std::isfinite(lr))
        return nfail(nullptr, SBLI_ERR_ARG, "sbli_adam_step: count >= 0, t >= 1 and lr > 0 required");
    if (count == 0) return SBLI_OK;
    adam_kernel<<<nblk(count), 256, 0, (hipStream_t)hip_stream>>>(p, g, m, v, count, lr, 0.9f, 0.999f, 1e-8f, t);
    return launch_status("sbli_adam_step");
}
