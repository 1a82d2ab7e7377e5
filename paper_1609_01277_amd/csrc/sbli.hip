// libsbli: host side of the C ABI declared in include/sbli.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/sbli.h"
#include "../../include/sbli_closure.h"
#include "kernels_pointwise.h"
#include "stage_variants.h"
#include "staged.h"
#include "stencil_weights.h"

using namespace sbli;

struct sbli_ctx {
    sbli_params p;
    hipStream_t stream;
    int device;
    int r;
    double h[3];
    double a[kMaxR], c0, c[kMaxR];
    BoxConst<double> c64;
    BoxConst<float> c32;
    int zchunk;             // z-planes per workgroup of the fused stage kernel
    int variant;            // index into the compiled stage variants of (dtype, order)
    BoxInst<double> inst64; // launch table entry (host copy) of the box
    BoxInst<float> inst32;
    void* inst_dev;         // the same entry on the device
    sbli_net* net;          // attached closure network (FP32 solvers) or null
    float* clos;            // closure term of the current stage (5 planar fields)
    int* cflag;             // guard verdict for clos
    unsigned* ccount;       // accepted / rejected closure evaluations
    double* diag_part;      // kDiagBlocks * (2 kDiagQ + 3)
    double* diag_da;        // 3 * kMaxR weights a_m / h (double) for the vorticity
    double* diag_out;       // 10 doubles
    void* stg;              // scratch of the staged form (kStagedScratchWords * P elements) or null
    std::string err;
};

static std::string g_init_err;

static int fail(sbli_ctx* ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_init_err = buf;
    return code;
}

#define HIP_TRY(ctx, call)                                                                          \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(ctx, SBLI_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
static void fill_const(const sbli_ctx* x, BoxConst<T>& c) {
    c.n[0] = x->p.nx;
    c.n[1] = x->p.ny;
    c.n[2] = x->p.nz;
    c.P = (int64_t)x->p.nx * x->p.ny * x->p.nz;
    for (int d = 0; d < 3; ++d) {
        for (int m = 0; m < kMaxR; ++m) {
            c.da[d][m] = (T)(m < x->r ? x->a[m] / x->h[d] : 0.0);
            c.d2c[d][m] = (T)(m < x->r ? x->c[m] / (x->h[d] * x->h[d]) : 0.0);
        }
        c.d2c0[d] = (T)(x->c0 / (x->h[d] * x->h[d]));
    }
    const double g = x->p.gamma, M = x->p.Mach;
    c.gm1 = (T)(g - 1.0);
    c.gM2 = (T)(g * M * M);
    c.inv_Re = (T)(1.0 / x->p.Re);
    c.inv_3Re = (T)(1.0 / (3.0 * x->p.Re));
    c.inv_Re23 = (T)(2.0 / (3.0 * x->p.Re));
    c.kappa = (T)(1.0 / ((g - 1.0) * M * M * x->p.Pr * x->p.Re));
    for (int d = 0; d < 3; ++d) c.sym[d] = x->p.bc[d] == SBLI_BC_SYMMETRY;
}

// z-planes per workgroup: long enough to amortise the 4R-plane pipeline fill,
// short enough to give the 256 compute units several workgroups each.
static int default_zchunk(const sbli_ctx* x) {
    const int tx = 16, ty = 16;
    const long tiles = (long)((x->p.nx + tx - 1) / tx) * ((x->p.ny + ty - 1) / ty);
    int zc = x->p.nz;
    while (zc > 32 && tiles * ((x->p.nz + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
    return zc;
}

// Variants of a context: the compiled fused variants of (dtype, order) (none
// beyond order 8), then the staged form (all fields of the StageVariant 0).
static int num_fused(const sbli_ctx* ctx) {
    if (ctx->r > 4) return 0;
    return ctx->p.dtype == SBLI_F64 ? StageDispatch<double>::count(ctx->r) : StageDispatch<float>::count(ctx->r);
}

static int num_variants(const sbli_ctx* ctx) { return num_fused(ctx) + 1; }

static bool is_staged(const sbli_ctx* ctx, int v) { return v == num_fused(ctx); }

static StageVariant variant_of(const sbli_ctx* ctx, int v) {
    if (is_staged(ctx, v)) return StageVariant{0, 0, 0, 0, 0, 0, 0};
    return ctx->p.dtype == SBLI_F64 ? StageDispatch<double>::get(ctx->r, v) : StageDispatch<float>::get(ctx->r, v);
}

static size_t elem_size(const sbli_ctx* x);
static int64_t npoints(const sbli_ctx* x);

// Allocates the staged form's scratch once (kept until sbli_destroy).
static hipError_t ensure_staged_scratch(sbli_ctx* x) {
    if (x->stg) return hipSuccess;
    return hipMalloc(&x->stg, (size_t)kStagedScratchWords * (size_t)npoints(x) * elem_size(x));
}

// Rebuilds the box's launch-table entry for the current variant and zchunk and
// copies it to the device, ordered on the context's stream, then waits for the
// copy so the host copy may change again.  The step time is 1 in the table;
// each launch passes the actual dt as its scale.
static hipError_t update_table(sbli_ctx* x) {
    if (is_staged(x, x->variant)) return ensure_staged_scratch(x);   // no launch table
    const StageVariant v = variant_of(x, x->variant);
    if (x->p.dtype == SBLI_F64) {
        x->inst64.c = x->c64;
        x->inst64.offset = 0;
        x->inst64.dt = 1.0;
        x->inst64.closure = nullptr;
        x->inst64.cflag = nullptr;
        set_box_geometry(x->inst64, v.tx, v.ty, x->zchunk, 0);
        hipError_t e = hipMemcpyAsync(x->inst_dev, &x->inst64, sizeof(x->inst64), hipMemcpyHostToDevice, x->stream);
        return e == hipSuccess ? hipStreamSynchronize(x->stream) : e;
    }
    x->inst32.c = x->c32;
    x->inst32.offset = 0;
    x->inst32.dt = 1.0f;
    x->inst32.closure = x->net ? x->clos : nullptr;
    x->inst32.cflag = x->net ? x->cflag : nullptr;
    set_box_geometry(x->inst32, v.tx, v.ty, x->zchunk, 0);
    hipError_t e = hipMemcpyAsync(x->inst_dev, &x->inst32, sizeof(x->inst32), hipMemcpyHostToDevice, x->stream);
    return e == hipSuccess ? hipStreamSynchronize(x->stream) : e;
}

static int total_wg(const sbli_ctx* x) { return x->p.dtype == SBLI_F64 ? x->inst64.num_wg : x->inst32.num_wg; }

static size_t elem_size(const sbli_ctx* x) { return x->p.dtype == SBLI_F32 ? sizeof(float) : sizeof(double); }
static int64_t npoints(const sbli_ctx* x) { return (int64_t)x->p.nx * x->p.ny * x->p.nz; }

static bool overlaps(const void* a, const void* b, size_t bytes) {
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    return pa < pb + bytes && pb < pa + bytes;
}

extern "C" int sbli_init(const sbli_params* p, void* hip_stream, sbli_ctx** out) {
    if (!out) return fail(nullptr, SBLI_ERR_ARG, "sbli_init: out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, SBLI_ERR_ARG, "sbli_init: params is NULL");
    if (p->order < 2 || p->order > 2 * kMaxR || p->order % 2 != 0)
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: order must be even, 2 to %d (got %d)", 2 * kMaxR, p->order);
    const int nmin = 2 * p->order + 1;
    if (p->nx < nmin || p->ny < nmin || p->nz < nmin)
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: every grid size must be >= %d for order %d (got %d x %d x %d)",
                    nmin, p->order, p->nx, p->ny, p->nz);
    if ((double)p->nx * p->ny * p->nz * 5.0 > 9.0e18)
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: grid too large");
    if (!(p->lx > 0 && p->ly > 0 && p->lz > 0 && std::isfinite(p->lx) && std::isfinite(p->ly) && std::isfinite(p->lz)))
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: box lengths must be finite and > 0");
    if (!(p->Re > 0 && p->Mach > 0 && p->Pr > 0 && std::isfinite(p->Re) && std::isfinite(p->Mach) && std::isfinite(p->Pr)))
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: Re, Mach and Pr must be finite and > 0");
    if (!(p->gamma > 1.0 && std::isfinite(p->gamma)))
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: gamma must be finite and > 1");
    if (p->dtype != SBLI_F64 && p->dtype != SBLI_F32)
        return fail(nullptr, SBLI_ERR_ARG, "sbli_init: dtype must be SBLI_F64 or SBLI_F32");
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] != SBLI_BC_PERIODIC && p->bc[d] != SBLI_BC_SYMMETRY)
            return fail(nullptr, SBLI_ERR_ARG, "sbli_init: bc[%d] must be SBLI_BC_PERIODIC or SBLI_BC_SYMMETRY (got %d)",
                        d, p->bc[d]);

    sbli_ctx* x = new (std::nothrow) sbli_ctx();
    if (!x) return fail(nullptr, SBLI_ERR_ALLOC, "sbli_init: out of host memory");
    x->p = *p;
    x->stream = (hipStream_t)hip_stream;
    x->r = p->order / 2;
    x->h[0] = p->lx / p->nx;
    x->h[1] = p->ly / p->ny;
    x->h[2] = p->lz / p->nz;
    central_weights(x->r, x->a, &x->c0, x->c);
    fill_const(x, x->c64);
    fill_const(x, x->c32);

    x->zchunk = default_zchunk(x);
    x->variant = 0;
    hipError_t e = hipGetDevice(&x->device);
    if (e == hipSuccess) e = hipMalloc((void**)&x->diag_part, sizeof(double) * kDiagBlocks * (2 * kDiagQ + 3));
    if (e == hipSuccess) e = hipMalloc((void**)&x->diag_da, sizeof(double) * 3 * kMaxR);
    if (e == hipSuccess) e = hipMalloc((void**)&x->diag_out, sizeof(double) * 10);
    if (e == hipSuccess) e = hipMalloc(&x->inst_dev, sizeof(BoxInst<double>));
    if (e == hipSuccess) e = update_table(x);
    if (e == hipSuccess) {
        double da[3 * kMaxR];
        for (int d = 0; d < 3; ++d)
            for (int m = 0; m < kMaxR; ++m) da[d * kMaxR + m] = m < x->r ? x->a[m] / x->h[d] : 0.0;
        e = hipMemcpyAsync(x->diag_da, da, sizeof(da), hipMemcpyHostToDevice, x->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
    }
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory) ? SBLI_ERR_ALLOC : SBLI_ERR_HIP;
        fail(nullptr, code, "sbli_init: %s", hipGetErrorString(e));
        // cleanup after the reported failure: its own status adds nothing
        (void)hipFree(x->diag_part);
        (void)hipFree(x->diag_da);
        (void)hipFree(x->diag_out);
        (void)hipFree(x->inst_dev);
        (void)hipFree(x->stg);
        delete x;
        return code;
    }
    *out = x;
    return SBLI_OK;
}

extern "C" int sbli_destroy(sbli_ctx* ctx) {
    if (!ctx) return SBLI_OK;
    // everything is released whatever fails; the first failure is reported
    hipError_t first = hipStreamSynchronize(ctx->stream);
    for (void* p : {(void*)ctx->diag_part, (void*)ctx->diag_da, (void*)ctx->diag_out, (void*)ctx->inst_dev, ctx->stg,
                    (void*)ctx->clos, (void*)ctx->cflag, (void*)ctx->ccount}) {
        const hipError_t e = hipFree(p);
        if (first == hipSuccess) first = e;
    }
    delete ctx;
    if (first != hipSuccess) return fail(nullptr, SBLI_ERR_HIP, "sbli_destroy: %s", hipGetErrorString(first));
    return SBLI_OK;
}

extern "C" const char* sbli_last_error(const sbli_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

extern "C" int sbli_tgv_init(sbli_ctx* ctx, void* q, const double* phase) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_tgv_init: ctx is NULL");
    if (!q) return fail(ctx, SBLI_ERR_ARG, "sbli_tgv_init: q is NULL");
    const double ph[3] = {phase ? phase[0] : 0.0, phase ? phase[1] : 0.0, phase ? phase[2] : 0.0};
    const int64_t P = npoints(ctx);
    const unsigned blocks = (unsigned)((P + 255) / 256);
    if (ctx->p.dtype == SBLI_F64)
        tgv_init_kernel<double><<<blocks, 256, 0, ctx->stream>>>((double*)q, ctx->p.nx, ctx->p.ny, ctx->p.nz, ctx->h[0],
                                                                 ctx->h[1], ctx->h[2], ph[0], ph[1], ph[2],
                                                                 ctx->p.gamma, ctx->p.Mach);
    else
        tgv_init_kernel<float><<<blocks, 256, 0, ctx->stream>>>((float*)q, ctx->p.nx, ctx->p.ny, ctx->p.nz, ctx->h[0],
                                                                ctx->h[1], ctx->h[2], ph[0], ph[1], ph[2],
                                                                ctx->p.gamma, ctx->p.Mach);
    HIP_TRY(ctx, hipGetLastError());
    return SBLI_OK;
}

// Enqueues one residual / stage launch of the selected variant.  The staged
// form's scratch exists whenever it is selected (update_table allocates it and
// a failed allocation leaves the previous variant selected); it is checked
// again here so that no launch ever runs without it.
static int launch_any(sbli_ctx* ctx, const void* qin, void* dq, void* qout, int mode, double dt, double A, double B) {
    if (is_staged(ctx, ctx->variant)) {
        if (!ctx->stg) return fail(ctx, SBLI_ERR_ALLOC, "stage launch: the staged form's scratch is not allocated");
        const bool f64 = ctx->p.dtype == SBLI_F64;
        const StagedArgs a{ctx->stream, f64, ctx->r, f64 ? (const void*)&ctx->c64 : (const void*)&ctx->c32,
                           ctx->stg, mode, dt, A, B, ctx->net ? ctx->clos : nullptr, ctx->net ? ctx->cflag : nullptr};
        staged_launch(a, qin, dq, qout);
        return SBLI_OK;
    }
    const int sym = ctx->p.bc[0] | ctx->p.bc[1] | ctx->p.bc[2];
    const StageArgs a{ctx->stream, ctx->inst_dev, 1, total_wg(ctx), mode, dt, A, B, sym};
    if (ctx->p.dtype == SBLI_F64)
        StageDispatch<double>::launch(ctx->r, ctx->variant, a, (const double*)qin, (double*)dq, (double*)qout);
    else
        StageDispatch<float>::launch(ctx->r, ctx->variant, a, (const float*)qin, (float*)dq, (float*)qout);
    return SBLI_OK;
}

extern "C" int sbli_rhs(sbli_ctx* ctx, const void* q, void* rhs) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_rhs: ctx is NULL");
    if (!q || !rhs) return fail(ctx, SBLI_ERR_ARG, "sbli_rhs: NULL state pointer");
    const size_t bytes = 5 * (size_t)npoints(ctx) * elem_size(ctx);
    if (overlaps(q, rhs, bytes)) return fail(ctx, SBLI_ERR_ARG, "sbli_rhs: q and rhs overlap");
    const int rc = launch_any(ctx, q, nullptr, rhs, kModeRHS, 0.0, 0.0, 0.0);
    if (rc != SBLI_OK) return rc;
    HIP_TRY(ctx, hipGetLastError());
    return SBLI_OK;
}

// Williamson's 2N-storage coefficients of the three-stage third-order scheme.
static const double kRK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double kRK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

// Enqueues nsteps RK3 steps ping-ponging between a and b; *result receives the
// buffer that holds the result.  Stops at the first failed call.
static int enqueue_steps(sbli_ctx* ctx, void* a, void* b, void* dq, double dt, int nsteps, void** result) {
    void* src = a;
    void* dst = b;
    *result = a;
    for (int s = 0; s < nsteps; ++s) {
        for (int k = 0; k < 3; ++k) {
            if (ctx->net) {
                // closure term of this stage's state, then its guard verdict (the
                // network enqueues on its own stream, which attach requires to be
                // the solver's)
                int rc = sbli_net_forward(ctx->net, (const float*)src, 1, ctx->clos);
                if (rc == SBLI_OK) rc = sbli_net_guard(ctx->net, ctx->clos, ctx->cflag, ctx->ccount);
                if (rc != SBLI_OK)
                    return fail(ctx, rc, "closure evaluation failed: %s", sbli_net_last_error(ctx->net));
            }
            const int rc = launch_any(ctx, src, dq, dst, kModeStage1 + k, dt, kRK_A[k], kRK_B[k]);
            if (rc != SBLI_OK) return rc;
            void* t = src;
            src = dst;
            dst = t;
        }
    }
    *result = src;
    return SBLI_OK;
}

extern "C" int sbli_rk3_step(sbli_ctx* ctx, void* q, void* q_tmp, void* dq, double dt, int nsteps) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_rk3_step: ctx is NULL");
    if (!q || !q_tmp || !dq) return fail(ctx, SBLI_ERR_ARG, "sbli_rk3_step: NULL state pointer");
    if (nsteps < 0) return fail(ctx, SBLI_ERR_ARG, "sbli_rk3_step: nsteps < 0");
    if (!std::isfinite(dt)) return fail(ctx, SBLI_ERR_ARG, "sbli_rk3_step: dt is not finite");
    const size_t bytes = 5 * (size_t)npoints(ctx) * elem_size(ctx);
    if (overlaps(q, q_tmp, bytes) || overlaps(q, dq, bytes) || overlaps(q_tmp, dq, bytes))
        return fail(ctx, SBLI_ERR_ARG, "sbli_rk3_step: q, q_tmp and dq must not overlap");
    void* src = q;
    const int rc = enqueue_steps(ctx, q, q_tmp, dq, dt, nsteps, &src);
    if (rc != SBLI_OK) return rc;
    HIP_TRY(ctx, hipGetLastError());
    if (src != q) HIP_TRY(ctx, hipMemcpyAsync(q, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    return SBLI_OK;
}

extern "C" int sbli_diagnostics(sbli_ctx* ctx, const void* q, double out[7]) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_diagnostics: ctx is NULL");
    if (!q || !out) return fail(ctx, SBLI_ERR_ARG, "sbli_diagnostics: NULL pointer");
    const int nb = kDiagBlocks;
    const double gm1 = ctx->p.gamma - 1.0;
    const int r = ctx->r;
#define DIAG_LAUNCH(T, RR)                                                                                      \
    diag_partial_kernel<T, RR><<<nb, DiagShape<RR>::NT, 0, ctx->stream>>>((const T*)q, ctx->p.nx, ctx->p.ny, ctx->p.nz, \
                                                                     ctx->diag_da, gm1, ctx->p.bc[0], ctx->p.bc[1], \
                                                                     ctx->p.bc[2], ctx->diag_part)
    if (ctx->p.dtype == SBLI_F64) {
        if (r == 1) DIAG_LAUNCH(double, 1); else if (r == 2) DIAG_LAUNCH(double, 2);
        else if (r == 3) DIAG_LAUNCH(double, 3); else if (r == 4) DIAG_LAUNCH(double, 4);
        else if (r == 5) DIAG_LAUNCH(double, 5); else DIAG_LAUNCH(double, 6);
    } else {
        if (r == 1) DIAG_LAUNCH(float, 1); else if (r == 2) DIAG_LAUNCH(float, 2);
        else if (r == 3) DIAG_LAUNCH(float, 3); else if (r == 4) DIAG_LAUNCH(float, 4);
        else if (r == 5) DIAG_LAUNCH(float, 5); else DIAG_LAUNCH(float, 6);
    }
#undef DIAG_LAUNCH
    HIP_TRY(ctx, hipGetLastError());
    diag_final_kernel<<<1, kDiagThreads, 0, ctx->stream>>>(ctx->diag_part, nb, 1.0 / (double)npoints(ctx), ctx->diag_out);
    HIP_TRY(ctx, hipGetLastError());
    double res[10];
    HIP_TRY(ctx, hipMemcpyAsync(res, ctx->diag_out, sizeof(res), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int d = 0; d < 7; ++d) out[d] = res[d];
    if (res[7] > 0 || res[8] > 0 || res[9] > 0)
        return fail(ctx, SBLI_ERR_NONFINITE, "sbli_diagnostics: %.0f non-finite values, %.0f points with rho <= 0, %.0f with p <= 0",
                    res[7], res[8], res[9]);
    return SBLI_OK;
}

extern "C" int sbli_num_variants(const sbli_ctx* ctx) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_num_variants: ctx is NULL");
    return num_variants(ctx);
}

extern "C" int sbli_variant_info(const sbli_ctx* ctx, int variant, int info[7]) {
    if (!ctx || !info) return fail(nullptr, SBLI_ERR_ARG, "sbli_variant_info: NULL argument");
    if (variant < 0 || variant >= num_variants(ctx))
        return fail(const_cast<sbli_ctx*>(ctx), SBLI_ERR_ARG, "sbli_variant_info: variant %d out of range", variant);
    const StageVariant v = variant_of(ctx, variant);
    info[0] = v.tx;
    info[1] = v.ty;
    info[2] = v.pre;
    info[3] = v.rot;
    info[4] = v.minw;
    info[5] = v.db;
    info[6] = v.zl;
    return SBLI_OK;
}

extern "C" int sbli_set_tuning(sbli_ctx* ctx, int variant, int zchunk) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_set_tuning: ctx is NULL");
    if (variant < 0 || variant >= num_variants(ctx))
        return fail(ctx, SBLI_ERR_ARG, "sbli_set_tuning: variant %d out of range [0, %d)", variant, num_variants(ctx));
    if (zchunk < 1 || zchunk > ctx->p.nz)
        return fail(ctx, SBLI_ERR_ARG, "sbli_set_tuning: zchunk %d out of range [1, %d]", zchunk, ctx->p.nz);
    const int old_v = ctx->variant, old_z = ctx->zchunk;
    ctx->variant = variant;
    ctx->zchunk = zchunk;
    const hipError_t e = update_table(ctx);
    if (e != hipSuccess) {
        ctx->variant = old_v;
        ctx->zchunk = old_z;
        (void)update_table(ctx);   // the previous configuration, rebuilt after the reported failure
        return fail(ctx, e == hipErrorOutOfMemory ? SBLI_ERR_ALLOC : SBLI_ERR_HIP, "sbli_set_tuning: %s",
                    hipGetErrorString(e));
    }
    return SBLI_OK;
}

extern "C" int sbli_get_tuning(const sbli_ctx* ctx, int* variant, int* zchunk) {
    if (!ctx || !variant || !zchunk) return fail(nullptr, SBLI_ERR_ARG, "sbli_get_tuning: NULL argument");
    *variant = ctx->variant;
    *zchunk = ctx->zchunk;
    return SBLI_OK;
}

// A later candidate replaces the best one only when it is faster by more than 1 %: candidates
// within timing noise of each other then resolve to the same (earlier) choice on every run.
constexpr float kTuneMargin = 0.99f;

extern "C" int sbli_autotune(sbli_ctx* ctx, void* q, void* q_tmp, void* dq, double dt, int reps, double* best_ms) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_autotune: ctx is NULL");
    if (!q || !q_tmp || !dq) return fail(ctx, SBLI_ERR_ARG, "sbli_autotune: NULL state pointer");
    if (reps < 1) return fail(ctx, SBLI_ERR_ARG, "sbli_autotune: reps must be >= 1");
    const size_t bytes = 5 * (size_t)npoints(ctx) * elem_size(ctx);
    if (overlaps(q, q_tmp, bytes) || overlaps(q, dq, bytes) || overlaps(q_tmp, dq, bytes))
        return fail(ctx, SBLI_ERR_ARG, "sbli_autotune: q, q_tmp and dq must not overlap");
    const int nz = ctx->p.nz;
    int cands[8], nc = 0;
    for (int zc = nz; zc >= 16 && nc < 6; zc = (zc + 1) / 2) {
        cands[nc++] = zc;
        if (zc == 16) break;
    }
    if (nc == 0) cands[nc++] = nz;
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    float best = 1e30f;
    int bv = ctx->variant, bz = ctx->zchunk;
    for (int v = 0; v < num_variants(ctx); ++v) {
        // the staged form has no z-chunks; it is skipped when its scratch cannot be allocated
        for (int ci = 0; ci < (is_staged(ctx, v) ? 1 : nc); ++ci) {
            ctx->variant = v;
            ctx->zchunk = cands[ci];
            if (update_table(ctx) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            void* res = nullptr;
            int rc = enqueue_steps(ctx, q, q_tmp, dq, dt, 1, &res);          // warm-up
            hipError_t err = hipEventRecord(e0, ctx->stream);
            if (rc == SBLI_OK && err == hipSuccess) rc = enqueue_steps(ctx, q, q_tmp, dq, dt, reps, &res);
            if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess && rc == SBLI_OK) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess || rc != SBLI_OK) {
                // cleanup after the failure reported below
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                ctx->variant = bv;
                ctx->zchunk = bz;
                (void)update_table(ctx);
                if (rc != SBLI_OK) return rc;
                return fail(ctx, SBLI_ERR_HIP, "sbli_autotune: %s", hipGetErrorString(err));
            }
            if (ms < best * kTuneMargin) {
                best = ms;
                bv = v;
                bz = cands[ci];
            }
        }
    }
    const hipError_t d0 = hipEventDestroy(e0), d1 = hipEventDestroy(e1);
    ctx->variant = bv;
    ctx->zchunk = bz;
    HIP_TRY(ctx, update_table(ctx));
    HIP_TRY(ctx, d0 != hipSuccess ? d0 : d1);
    if (best_ms) *best_ms = best / reps;
    return SBLI_OK;
}

// ---------------------------------------------------------------------------
// Ensembles: many periodic boxes (uneven sizes and parameters) stepped by one
// stage launch each, optionally recorded once into a hipGraph.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) copy_kernel(const T* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

struct sbli_batch {
    int count = 0, order = 4, dtype = SBLI_F64, r = 2;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;              // internal stream used only for graph capture
    std::vector<sbli_ctx*> ctx;             // one context per box (constants, diagnostics scratch)
    std::vector<sbli_instance> inst;
    std::vector<size_t> off;                // element offsets, count + 1 entries
    int variant = 0, zmax = 64;
    std::vector<BoxInst<double>> t64;
    std::vector<BoxInst<float>> t32;
    void* table_dev = nullptr;
    int total_wg = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

static std::string g_batch_err;

static int bfail(sbli_batch* b, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_batch_err = buf;
    return code;
}

#define BHIP_TRY(b, call)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return bfail(b, SBLI_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t belem(const sbli_batch* b) { return b->dtype == SBLI_F32 ? sizeof(float) : sizeof(double); }

// Releases the captured graph; returns the first failure of the two releases.
static hipError_t batch_drop_graph(sbli_batch* b) {
    hipError_t e = hipSuccess;
    if (b->exec) e = hipGraphExecDestroy(b->exec);
    if (b->graph) {
        const hipError_t e2 = hipGraphDestroy(b->graph);
        if (e == hipSuccess) e = e2;
    }
    b->exec = nullptr;
    b->graph = nullptr;
    return e;
}

// Rebuilds the launch table for the current variant and z-chunk cap, copies it
// to the device (waiting for the copy) and gives every per-box context the same
// launch configuration, so box-by-box stepping runs the same kernels.
static int batch_build_table(sbli_batch* b) {
    const StageVariant v = b->dtype == SBLI_F64 ? StageDispatch<double>::get(b->r, b->variant)
                                                : StageDispatch<float>::get(b->r, b->variant);
    int first = 0;
    b->t64.assign(b->count, BoxInst<double>{});
    b->t32.assign(b->count, BoxInst<float>{});
    for (int i = 0; i < b->count; ++i) {
        const int zc = std::min(b->inst[i].n, b->zmax);
        if (b->dtype == SBLI_F64) {
            BoxInst<double>& e = b->t64[i];
            e.c = b->ctx[i]->c64;
            e.offset = (int64_t)b->off[i];
            e.dt = b->inst[i].dt;
            first += set_box_geometry(e, v.tx, v.ty, zc, first);
        } else {
            BoxInst<float>& e = b->t32[i];
            e.c = b->ctx[i]->c32;
            e.offset = (int64_t)b->off[i];
            e.dt = (float)b->inst[i].dt;
            first += set_box_geometry(e, v.tx, v.ty, zc, first);
        }
        int rc = sbli_set_tuning(b->ctx[i], b->variant, zc);
        if (rc != SBLI_OK) return bfail(b, rc, "batch: %s", sbli_last_error(b->ctx[i]));
    }
    b->total_wg = first;
    const void* src = b->dtype == SBLI_F64 ? (const void*)b->t64.data() : (const void*)b->t32.data();
    const size_t bytes = b->dtype == SBLI_F64 ? sizeof(BoxInst<double>) * b->count : sizeof(BoxInst<float>) * b->count;
    BHIP_TRY(b, hipMemcpyAsync(b->table_dev, src, bytes, hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    BHIP_TRY(b, batch_drop_graph(b));
    return SBLI_OK;
}

static void batch_launch_stage(sbli_batch* b, hipStream_t s, const void* qin, void* dq, void* qout, int k) {
    const StageArgs a{s, b->table_dev, b->count, b->total_wg, kModeStage1 + k, 1.0, kRK_A[k], kRK_B[k], 0};
    if (b->dtype == SBLI_F64)
        StageDispatch<double>::launch(b->r, b->variant, a, (const double*)qin, (double*)dq, (double*)qout);
    else
        StageDispatch<float>::launch(b->r, b->variant, a, (const float*)qin, (float*)dq, (float*)qout);
}

// nsteps steps of every box, 3 launches per step; a final copy kernel puts the
// result back in q when it ended in q_tmp.
static void batch_enqueue(sbli_batch* b, hipStream_t s, void* q, void* q_tmp, void* dq, int nsteps) {
    void* src = q;
    void* dst = q_tmp;
    for (int st = 0; st < nsteps; ++st)
        for (int k = 0; k < 3; ++k) {
            batch_launch_stage(b, s, src, dq, dst, k);
            std::swap(src, dst);
        }
    if (src != q) {
        const int64_t n = (int64_t)b->off[b->count];
        const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
        if (b->dtype == SBLI_F64) copy_kernel<double><<<blocks, 256, 0, s>>>((const double*)src, (double*)q, n);
        else copy_kernel<float><<<blocks, 256, 0, s>>>((const float*)src, (float*)q, n);
    }
}

static int batch_check_buffers(sbli_batch* b, const char* who, void* q, void* q_tmp, void* dq) {
    if (!q || !q_tmp || !dq) return bfail(b, SBLI_ERR_ARG, "%s: NULL state pointer", who);
    const size_t bytes = b->off[b->count] * belem(b);
    if (overlaps(q, q_tmp, bytes) || overlaps(q, dq, bytes) || overlaps(q_tmp, dq, bytes))
        return bfail(b, SBLI_ERR_ARG, "%s: q, q_tmp and dq must not overlap", who);
    return SBLI_OK;
}

extern "C" int sbli_batch_destroy(sbli_batch* b) {
    if (!b) return SBLI_OK;
    // everything is released whatever fails; the first failure is reported
    hipError_t first = hipStreamSynchronize(b->stream);
    auto keep = [&](hipError_t e) {
        if (first == hipSuccess) first = e;
    };
    keep(batch_drop_graph(b));
    if (b->cap) keep(hipStreamDestroy(b->cap));
    keep(hipFree(b->table_dev));
    int rc = SBLI_OK;
    for (sbli_ctx* c : b->ctx) {
        const int r = sbli_destroy(c);
        if (rc == SBLI_OK) rc = r;
    }
    delete b;
    if (first != hipSuccess) return bfail(nullptr, SBLI_ERR_HIP, "sbli_batch_destroy: %s", hipGetErrorString(first));
    if (rc != SBLI_OK) return bfail(nullptr, rc, "sbli_batch_destroy: %s", sbli_last_error(nullptr));
    return SBLI_OK;
}

extern "C" const char* sbli_batch_last_error(const sbli_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

extern "C" int sbli_batch_init(const sbli_instance* inst, int count, int order, int dtype, void* hip_stream,
                               sbli_batch** out) {
    if (!out) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_init: out is NULL");
    *out = nullptr;
    if (!inst || count < 1) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_init: need count >= 1 instances");
    // one launch covers all boxes: only the fused stage kernel (orders 2..8) takes a box table
    if (order != 2 && order != 4 && order != 6 && order != 8)
        return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_init: order must be 2, 4, 6 or 8 (got %d)", order);
    for (int i = 0; i < count; ++i)
        if (!(inst[i].dt > 0 && std::isfinite(inst[i].dt)))
            return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_init: instance %d: dt must be finite and > 0", i);
    sbli_batch* b = new (std::nothrow) sbli_batch();
    if (!b) return bfail(nullptr, SBLI_ERR_ALLOC, "sbli_batch_init: out of host memory");
    b->count = count;
    b->order = order;
    b->dtype = dtype;
    b->r = order / 2;
    b->stream = (hipStream_t)hip_stream;
    b->inst.assign(inst, inst + count);
    b->off.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        sbli_params p{inst[i].n, inst[i].n, inst[i].n, 2 * M_PI, 2 * M_PI, 2 * M_PI, inst[i].Re, inst[i].Mach,
                      inst[i].Pr, inst[i].gamma, order, dtype};
        sbli_ctx* c = nullptr;
        int rc = sbli_init(&p, hip_stream, &c);
        if (rc != SBLI_OK) {
            bfail(nullptr, rc, "sbli_batch_init: instance %d: %s", i, sbli_last_error(nullptr));
            sbli_batch_destroy(b);
            return rc;
        }
        b->ctx.push_back(c);
        b->off[i + 1] = b->off[i] + 5 * (size_t)inst[i].n * inst[i].n * inst[i].n;
    }
    hipError_t e = hipMalloc(&b->table_dev, sizeof(BoxInst<double>) * count);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        bfail(nullptr, SBLI_ERR_HIP, "sbli_batch_init: %s", hipGetErrorString(e));
        sbli_batch_destroy(b);
        return SBLI_ERR_HIP;
    }
    int rc = batch_build_table(b);
    if (rc != SBLI_OK) {
        g_batch_err = b->err;
        sbli_batch_destroy(b);
        return rc;
    }
    *out = b;
    return SBLI_OK;
}

extern "C" int sbli_batch_layout(const sbli_batch* b, size_t* offsets) {
    if (!b || !offsets) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_layout: NULL argument");
    for (int i = 0; i <= b->count; ++i) offsets[i] = b->off[i];
    return SBLI_OK;
}

extern "C" int sbli_batch_tgv_init(sbli_batch* b, void* q) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_tgv_init: batch is NULL");
    if (!q) return bfail(b, SBLI_ERR_ARG, "sbli_batch_tgv_init: q is NULL");
    for (int i = 0; i < b->count; ++i) {
        int rc = sbli_tgv_init(b->ctx[i], (char*)q + b->off[i] * belem(b), b->inst[i].phase);
        if (rc != SBLI_OK) return bfail(b, rc, "sbli_batch_tgv_init: %s", sbli_last_error(b->ctx[i]));
    }
    return SBLI_OK;
}

extern "C" int sbli_batch_step(sbli_batch* b, void* q, void* q_tmp, void* dq, int nsteps) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_step: batch is NULL");
    int rc = batch_check_buffers(b, "sbli_batch_step", q, q_tmp, dq);
    if (rc != SBLI_OK) return rc;
    if (nsteps < 0) return bfail(b, SBLI_ERR_ARG, "sbli_batch_step: nsteps < 0");
    batch_enqueue(b, b->stream, q, q_tmp, dq, nsteps);
    BHIP_TRY(b, hipGetLastError());
    return SBLI_OK;
}

extern "C" int sbli_batch_step_sequential(sbli_batch* b, void* q, void* q_tmp, void* dq, int nsteps) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_step_sequential: batch is NULL");
    int rc = batch_check_buffers(b, "sbli_batch_step_sequential", q, q_tmp, dq);
    if (rc != SBLI_OK) return rc;
    if (nsteps < 0) return bfail(b, SBLI_ERR_ARG, "sbli_batch_step_sequential: nsteps < 0");
    const size_t es = belem(b);
    for (int i = 0; i < b->count; ++i) {
        rc = sbli_rk3_step(b->ctx[i], (char*)q + b->off[i] * es, (char*)q_tmp + b->off[i] * es,
                           (char*)dq + b->off[i] * es, b->inst[i].dt, nsteps);
        if (rc != SBLI_OK) return bfail(b, rc, "sbli_batch_step_sequential: %s", sbli_last_error(b->ctx[i]));
    }
    return SBLI_OK;
}

extern "C" int sbli_batch_capture(sbli_batch* b, void* q, void* q_tmp, void* dq, int nsteps) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_capture: batch is NULL");
    int rc = batch_check_buffers(b, "sbli_batch_capture", q, q_tmp, dq);
    if (rc != SBLI_OK) return rc;
    if (nsteps < 1) return bfail(b, SBLI_ERR_ARG, "sbli_batch_capture: nsteps must be >= 1");
    BHIP_TRY(b, batch_drop_graph(b));
    BHIP_TRY(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    batch_enqueue(b, b->cap, q, q_tmp, dq, nsteps);
    hipError_t le = hipGetLastError();
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);   // cleanup after the failure reported here
        return bfail(b, SBLI_ERR_HIP, "sbli_batch_capture: %s",
                     hipGetErrorString(le != hipSuccess ? le : ce));
    }
    b->graph = g;
    hipError_t ie = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)batch_drop_graph(b);   // cleanup after the failure reported here
        return bfail(b, SBLI_ERR_HIP, "sbli_batch_capture: hipGraphInstantiate: %s", hipGetErrorString(ie));
    }
    return SBLI_OK;
}

extern "C" int sbli_batch_launch(sbli_batch* b) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_launch: batch is NULL");
    if (!b->exec) return bfail(b, SBLI_ERR_ARG, "sbli_batch_launch: nothing captured (call sbli_batch_capture)");
    BHIP_TRY(b, hipGraphLaunch(b->exec, b->stream));
    return SBLI_OK;
}

extern "C" int sbli_batch_diagnostics(sbli_batch* b, const void* q, double* out) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_diagnostics: batch is NULL");
    if (!q || !out) return bfail(b, SBLI_ERR_ARG, "sbli_batch_diagnostics: NULL pointer");
    int status = SBLI_OK;
    for (int i = 0; i < b->count; ++i) {
        int rc = sbli_diagnostics(b->ctx[i], (const char*)q + b->off[i] * belem(b), out + 7 * i);
        if (rc == SBLI_ERR_NONFINITE) {
            status = rc;
            bfail(b, rc, "sbli_batch_diagnostics: instance %d: %s", i, sbli_last_error(b->ctx[i]));
        } else if (rc != SBLI_OK) {
            return bfail(b, rc, "sbli_batch_diagnostics: instance %d: %s", i, sbli_last_error(b->ctx[i]));
        }
    }
    return status;
}

extern "C" int sbli_batch_set_tuning(sbli_batch* b, int variant, int zmax) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_set_tuning: batch is NULL");
    const int nv = b->dtype == SBLI_F64 ? StageDispatch<double>::count(b->r) : StageDispatch<float>::count(b->r);
    if (variant < 0 || variant >= nv)
        return bfail(b, SBLI_ERR_ARG, "sbli_batch_set_tuning: variant %d out of range [0, %d)", variant, nv);
    if (zmax < 1) return bfail(b, SBLI_ERR_ARG, "sbli_batch_set_tuning: zmax must be >= 1");
    b->variant = variant;
    b->zmax = zmax;
    return batch_build_table(b);
}

extern "C" int sbli_batch_get_tuning(const sbli_batch* b, int* variant, int* zmax) {
    if (!b || !variant || !zmax) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_get_tuning: NULL argument");
    *variant = b->variant;
    *zmax = b->zmax;
    return SBLI_OK;
}

extern "C" int sbli_batch_autotune(sbli_batch* b, void* q, void* q_tmp, void* dq, int reps, double* best_ms) {
    if (!b) return bfail(nullptr, SBLI_ERR_ARG, "sbli_batch_autotune: batch is NULL");
    int rc = batch_check_buffers(b, "sbli_batch_autotune", q, q_tmp, dq);
    if (rc != SBLI_OK) return rc;
    if (reps < 1) return bfail(b, SBLI_ERR_ARG, "sbli_batch_autotune: reps must be >= 1");
    const int nv = b->dtype == SBLI_F64 ? StageDispatch<double>::count(b->r) : StageDispatch<float>::count(b->r);
    const int zc[6] = {128, 96, 64, 48, 32, 16};
    hipEvent_t e0, e1;
    BHIP_TRY(b, hipEventCreate(&e0));
    BHIP_TRY(b, hipEventCreate(&e1));
    float best = 1e30f;
    int bv = b->variant, bz = b->zmax;
    hipError_t err = hipSuccess;
    // a failure ends both loops; rc and err then hold it
    for (int v = 0; v < nv && rc == SBLI_OK && err == hipSuccess; ++v)
        for (int zi = 0; zi < 6; ++zi) {
            b->variant = v;
            b->zmax = zc[zi];
            rc = batch_build_table(b);
            if (rc != SBLI_OK) break;
            batch_enqueue(b, b->stream, q, q_tmp, dq, 1);
            err = hipGetLastError();
            if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
            if (err == hipSuccess) {
                batch_enqueue(b, b->stream, q, q_tmp, dq, reps);
                err = hipGetLastError();
            }
            if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess) break;
            if (ms < best * kTuneMargin) {
                best = ms;
                bv = v;
                bz = zc[zi];
            }
        }
    const hipError_t d0 = hipEventDestroy(e0), d1 = hipEventDestroy(e1);
    if (err == hipSuccess) err = d0 != hipSuccess ? d0 : d1;
    b->variant = bv;
    b->zmax = bz;
    const int rc2 = batch_build_table(b);
    if (rc != SBLI_OK) return rc;   // batch_build_table has recorded the message
    if (err != hipSuccess) return bfail(b, SBLI_ERR_HIP, "sbli_batch_autotune: %s", hipGetErrorString(err));
    if (rc2 != SBLI_OK) return rc2;
    if (best_ms) *best_ms = best / reps;
    return SBLI_OK;
}

extern "C" int sbli_closure_attach(sbli_ctx* ctx, sbli_net* net) {
    if (!ctx) return fail(nullptr, SBLI_ERR_ARG, "sbli_closure_attach: ctx is NULL");
    if (net) {
        if (ctx->p.dtype != SBLI_F32)
            return fail(ctx, SBLI_ERR_ARG, "sbli_closure_attach: the closure needs an FP32 solver");
        const int n = sbli_net_n(net);
        if (ctx->p.nx != n || ctx->p.ny != n || ctx->p.nz != n)
            return fail(ctx, SBLI_ERR_ARG, "sbli_closure_attach: grid %dx%dx%d does not match the network's %d^3",
                        ctx->p.nx, ctx->p.ny, ctx->p.nz, n);
        if (sbli_net_stream(net) != (void*)ctx->stream)
            return fail(ctx, SBLI_ERR_ARG,
                        "sbli_closure_attach: the network and the solver must use the same HIP stream "
                        "(the stage kernel reads the closure term that the network writes)");
        if (!ctx->clos) {
            HIP_TRY(ctx, hipMalloc((void**)&ctx->clos, sizeof(float) * 5 * (size_t)npoints(ctx)));
            HIP_TRY(ctx, hipMalloc((void**)&ctx->cflag, sizeof(int)));
            HIP_TRY(ctx, hipMalloc((void**)&ctx->ccount, 2 * sizeof(unsigned)));
            HIP_TRY(ctx, hipMemsetAsync(ctx->ccount, 0, 2 * sizeof(unsigned), ctx->stream));
        }
    }
    ctx->net = net;
    HIP_TRY(ctx, update_table(ctx));
    return SBLI_OK;
}

extern "C" int sbli_closure_counts(sbli_ctx* ctx, unsigned counts[2]) {
    if (!ctx || !counts) return fail(ctx, SBLI_ERR_ARG, "sbli_closure_counts: NULL argument");
    counts[0] = counts[1] = 0;
    if (!ctx->ccount) return SBLI_OK;
    HIP_TRY(ctx, hipMemcpyAsync(counts, ctx->ccount, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return SBLI_OK;
}
