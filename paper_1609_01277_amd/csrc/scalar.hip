// libsbli: scalar advection-diffusion on a periodic grid (include/sbli_scalar.h),
// the equation of the paper's 1D wave and 2D manufactured-solution cases, on the
// same central stencils (any even order 2..12) and the same low-storage RK3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/sbli.h"
#include "../../include/sbli_scalar.h"
#include "sbli_common.h"
#include "stencil_weights.h"

using namespace sbli;

namespace {

constexpr int kScalarMaxR = 6;

struct ScalarConst {
    int n[3];
    int64_t P;
    int r;
    int active[3];                  // axes with more than one point
    double da[3][kScalarMaxR];      // a_m / h
    double d2c0[3];                 // c_0 / h^2
    double d2c[3][kScalarMaxR];     // c_m / h^2
    double c[3];                    // advection velocity
    double k;                       // diffusivity
};

// Index of the neighbour m points away on a periodic axis of n points, for any m
// (a stencil may be wider than the grid: indices wrap modulo n).
__device__ __forceinline__ int64_t wrapped(int64_t id, int c, int m, int n, int64_t stride) {
    unsigned flip;
    const int cc = fold_index(c + m, n, 0, flip);
    return id + (int64_t)(cc - c) * stride;
}

// R = -sum_j c_j D_j phi + k sum_j D2_j phi - S, then (MODE != RHS) the 2N stage
// dq <- A dq + dt R, out <- phi + B dq.  One thread per point; neighbours through
// the caches (a scalar field needs no LDS staging to stay memory-bound).
template <int MODE>
__global__ void __launch_bounds__(256) scalar_stage_kernel(const double* __restrict__ phi,
                                                           const double* __restrict__ S, double* __restrict__ dq,
                                                           double* __restrict__ out, ScalarConst c, double dt,
                                                           double A, double B) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= c.P) return;
    const int i = (int)(id % c.n[0]);
    const int64_t t = id / c.n[0];
    const int j = (int)(t % c.n[1]);
    const int k = (int)(t / c.n[1]);
    const int coord[3] = {i, j, k};
    const int64_t stride[3] = {1, (int64_t)c.n[0], (int64_t)c.n[0] * c.n[1]};
    const double f0 = phi[id];
    double R = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (!c.active[d]) continue;
        double s1 = 0.0, s2 = c.d2c0[d] * f0;
        for (int m = 1; m <= c.r; ++m) {
            const double fp = phi[wrapped(id, coord[d], m, c.n[d], stride[d])];
            const double fm = phi[wrapped(id, coord[d], -m, c.n[d], stride[d])];
            s1 += c.da[d][m - 1] * (fp - fm);
            s2 += c.d2c[d][m - 1] * (fp + fm);
        }
        R += c.k * s2 - c.c[d] * s1;
    }
    if (S) R -= S[id];
    if (MODE == kModeRHS) {
        out[id] = R;
    } else {
        double dn = dt * R;
        if (MODE != kModeStage1) dn += A * dq[id];
        if (MODE != kModeStage3) dq[id] = dn;
        out[id] = f0 + B * dn;
    }
}

__global__ void __launch_bounds__(256) scalar_copy_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                          int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

thread_local std::string t_err;

int sfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

int make_const(const sbli_scalar_params* p, ScalarConst* c) {
    if (!p) return sfail(SBLI_ERR_ARG, "scalar: params is NULL");
    if (p->order < 2 || p->order > 2 * kScalarMaxR || p->order % 2)
        return sfail(SBLI_ERR_ARG, "scalar: order must be even in [2, %d] (got %d)", 2 * kScalarMaxR, p->order);
    const int r = p->order / 2;
    double a[kScalarMaxR], cc[kScalarMaxR], c0;
    central_weights(r, a, &c0, cc);
    c->r = r;
    c->P = 1;
    int nact = 0;
    for (int d = 0; d < 3; ++d) {
        const int n = p->n[d];
        if (n < 1) return sfail(SBLI_ERR_ARG, "scalar: n[%d] must be >= 1", d);
        c->n[d] = n;
        c->P *= n;
        c->active[d] = n > 1;
        nact += n > 1;
        if (n > 1 && !(p->length[d] > 0 && std::isfinite(p->length[d])))
            return sfail(SBLI_ERR_ARG, "scalar: length[%d] must be finite and > 0", d);
        const double h = n > 1 ? p->length[d] / n : 1.0;
        for (int m = 0; m < kScalarMaxR; ++m) {
            c->da[d][m] = m < r ? a[m] / h : 0.0;
            c->d2c[d][m] = m < r ? cc[m] / (h * h) : 0.0;
        }
        c->d2c0[d] = c0 / (h * h);
        c->c[d] = p->c[d];
        if (!std::isfinite(p->c[d])) return sfail(SBLI_ERR_ARG, "scalar: velocity must be finite");
    }
    if (nact == 0) return sfail(SBLI_ERR_ARG, "scalar: at least one axis needs more than one point");
    if (!(p->k >= 0 && std::isfinite(p->k))) return sfail(SBLI_ERR_ARG, "scalar: k must be finite and >= 0");
    c->k = p->k;
    return SBLI_OK;
}

const double kA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double kB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

}  // namespace

extern "C" const char* sbli_scalar_last_error(void) { return t_err.c_str(); }

extern "C" int sbli_scalar_rhs(const sbli_scalar_params* p, const double* phi, const double* source, double* rhs,
                               void* hip_stream) {
    ScalarConst c;
    int rc = make_const(p, &c);
    if (rc != SBLI_OK) return rc;
    if (!phi || !rhs) return sfail(SBLI_ERR_ARG, "sbli_scalar_rhs: NULL pointer");
    if (phi == rhs) return sfail(SBLI_ERR_ARG, "sbli_scalar_rhs: phi and rhs must differ");
    const unsigned blocks = (unsigned)((c.P + 255) / 256);
    scalar_stage_kernel<kModeRHS><<<blocks, 256, 0, (hipStream_t)hip_stream>>>(phi, source, nullptr, rhs, c, 0.0,
                                                                              0.0, 0.0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sfail(SBLI_ERR_HIP, "sbli_scalar_rhs: %s", hipGetErrorString(e));
    return SBLI_OK;
}

extern "C" int sbli_scalar_rk3(const sbli_scalar_params* p, double* phi, double* phi_tmp, double* dphi,
                               const double* source, double dt, int nsteps, void* hip_stream) {
    ScalarConst c;
    int rc = make_const(p, &c);
    if (rc != SBLI_OK) return rc;
    if (!phi || !phi_tmp || !dphi) return sfail(SBLI_ERR_ARG, "sbli_scalar_rk3: NULL pointer");
    if (phi == phi_tmp || phi == dphi || phi_tmp == dphi)
        return sfail(SBLI_ERR_ARG, "sbli_scalar_rk3: phi, phi_tmp and dphi must be distinct");
    if (nsteps < 0 || !std::isfinite(dt)) return sfail(SBLI_ERR_ARG, "sbli_scalar_rk3: need nsteps >= 0, finite dt");
    hipStream_t s = (hipStream_t)hip_stream;
    const unsigned blocks = (unsigned)((c.P + 255) / 256);
    double* src = phi;
    double* dst = phi_tmp;
    for (int st = 0; st < nsteps; ++st) {
        scalar_stage_kernel<kModeStage1><<<blocks, 256, 0, s>>>(src, source, dphi, dst, c, dt, kA[0], kB[0]);
        std::swap(src, dst);
        scalar_stage_kernel<kModeStage2><<<blocks, 256, 0, s>>>(src, source, dphi, dst, c, dt, kA[1], kB[1]);
        std::swap(src, dst);
        scalar_stage_kernel<kModeStage3><<<blocks, 256, 0, s>>>(src, source, dphi, dst, c, dt, kA[2], kB[2]);
        std::swap(src, dst);
    }
    if (src != phi) {
        const unsigned cb = (unsigned)std::min<int64_t>((c.P + 255) / 256, 65536);
        scalar_copy_kernel<<<cb, 256, 0, s>>>(src, phi, c.P);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sfail(SBLI_ERR_HIP, "sbli_scalar_rk3: %s", hipGetErrorString(e));
    return SBLI_OK;
}
