// Point-per-thread residual and RK3-stage kernels (neighbours read through the
// caches).  Two launches per stage: grad_kernel writes the six fields that the
// nested (outer) derivatives act on, stage_kernel does everything else.
#pragma once

#include "sbli_common.h"

namespace sbli {

// Inner derivatives of the nested terms (paper Sec. "Expanding": the inner
// derivative is evaluated first, then the outer one).  With g_ij = D_j u_i,
// theta = g_kk and tau_ij = (1/Re)(g_ij + g_ji - 2/3 delta_ij theta):
//   W[j]     = V_j = sum_i u_i tau_ij     (viscous work flux)
//   W[3 + i] = theta - g_ii               (= sum_{k != i} D_k u_k)
template <typename T, int R>
__global__ void __launch_bounds__(256) grad_kernel(const T* __restrict__ q, T* __restrict__ W, BoxConst<T> c) {
    const int64_t P = c.P;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= P) return;
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int i = (int)(id % nx);
    const int64_t t = id / nx;
    const int j = (int)(t % ny);
    const int k = (int)(t / ny);
    const int coord[3] = {i, j, k};
    const int64_t strides[3] = {1, (int64_t)nx, (int64_t)nx * ny};
    T g[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
            const int64_t ip = shifted(id, coord[a], m, c.n[a], strides[a]);
            const int64_t im = shifted(id, coord[a], -m, c.n[a], strides[a]);
            const T rp = T(1) / q[ip], rm = T(1) / q[im];
            const T w = c.da[a][m - 1];
            s0 += w * (q[P + ip] * rp - q[P + im] * rm);
            s1 += w * (q[2 * P + ip] * rp - q[2 * P + im] * rm);
            s2 += w * (q[3 * P + ip] * rp - q[3 * P + im] * rm);
        }
        g[0][a] = s0;
        g[1][a] = s1;
        g[2][a] = s2;
    }
    const T rr = T(1) / q[id];
    const T u[3] = {q[P + id] * rr, q[2 * P + id] * rr, q[3 * P + id] * rr};
    const T theta = g[0][0] + g[1][1] + g[2][2];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
        T v = 0;
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
            T tau = c.inv_Re * (g[ii][jj] + g[jj][ii]);
            if (ii == jj) tau -= c.inv_Re23 * theta;
            v += u[ii] * tau;
        }
        W[jj * P + id] = v;
        W[(3 + jj) * P + id] = theta - g[jj][jj];
    }
}

// Pointwise primitive variables of a state value.
template <typename T>
struct Prim {
    T rho, m[3], E, u[3], p, Tm;
};

template <typename T>
__device__ __forceinline__ Prim<T> load_prim(const T* __restrict__ q, int64_t P, int64_t id, const BoxConst<T>& c) {
    Prim<T> s;
    s.rho = q[id];
    s.m[0] = q[P + id];
    s.m[1] = q[2 * P + id];
    s.m[2] = q[3 * P + id];
    s.E = q[4 * P + id];
    const T rr = T(1) / s.rho;
    s.u[0] = s.m[0] * rr;
    s.u[1] = s.m[1] * rr;
    s.u[2] = s.m[2] * rr;
    s.p = c.gm1 * (s.E - T(0.5) * (s.m[0] * s.u[0] + s.m[1] * s.u[1] + s.m[2] * s.u[2]));
    s.Tm = c.gM2 * s.p * rr;
    return s;
}

enum StageMode { kModeRHS = 0, kModeStage1 = 1, kModeStage2 = 2, kModeStage3 = 3 };

// Residual (paper eq. mass, momentum, energy with the skew-symmetric convective
// form) grouped by direction j, then either stored (kModeRHS) or applied as one
// stage of the 2N RK3 scheme:  dq <- A dq + dt R;  q_out <- q_in + B dq.
// Per direction j the derivatives taken are
//   D_j rho, D_j(rho u_i), D_j(rho u_i u_j + 2 p delta_ij), D_j(rho E),
//   D_j((rho E + 2p) u_j - 2 V_j), D_j u_j, D2_j u_i, D2_j T, D_j(theta - g_jj)
// which regroup the paper's terms by linearity:
//   -1/2 D_j(2 p delta_ij) = -D_i p, and
//   -1/2 D_j((rho E + 2 p) u_j - 2 V_j) = -1/2 D_j(rho E u_j) - D_j(p u_j) + D_j(u_i tau_ij).
template <typename T, int R, int MODE>
__global__ void __launch_bounds__(256) stage_kernel(const T* __restrict__ q, const T* __restrict__ W,
                                                     T* __restrict__ dq, T* __restrict__ out, BoxConst<T> c,
                                                     T dt, T A, T B) {
    const int64_t P = c.P;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= P) return;
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int i = (int)(id % nx);
    const int64_t t = id / nx;
    const int j = (int)(t % ny);
    const int k = (int)(t / ny);
    const int coord[3] = {i, j, k};
    const int64_t strides[3] = {1, (int64_t)nx, (int64_t)nx * ny};
    const Prim<T> s = load_prim(q, P, id, c);

    T Rr = 0, Rm[3] = {0, 0, 0}, RE = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T dRho = 0, dM[3] = {0, 0, 0}, dF[3] = {0, 0, 0}, dE = 0, dH = 0, dU = 0, dTh = 0;
        T d2U[3] = {0, 0, 0}, d2T = 0;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
            const int64_t ip = shifted(id, coord[d], m, c.n[d], strides[d]);
            const int64_t im = shifted(id, coord[d], -m, c.n[d], strides[d]);
            const Prim<T> a = load_prim(q, P, ip, c);
            const Prim<T> b = load_prim(q, P, im, c);
            const T Va = W[d * P + ip], Vb = W[d * P + im];
            const T Ta = W[(3 + d) * P + ip], Tb = W[(3 + d) * P + im];
            const T w = c.da[d][m - 1], w2 = c.d2c[d][m - 1];
            dRho += w * (a.rho - b.rho);
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                dM[e] += w * (a.m[e] - b.m[e]);
                T fa = a.m[e] * a.u[d], fb = b.m[e] * b.u[d];
                if (e == d) { fa += T(2) * a.p; fb += T(2) * b.p; }
                dF[e] += w * (fa - fb);
                d2U[e] += w2 * (a.u[e] + b.u[e]);
            }
            dE += w * (a.E - b.E);
            dH += w * (((a.E + T(2) * a.p) * a.u[d] - T(2) * Va) - ((b.E + T(2) * b.p) * b.u[d] - T(2) * Vb));
            dU += w * (a.u[d] - b.u[d]);
            dTh += w * (Ta - Tb);
            d2T += w2 * (a.Tm + b.Tm);
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) d2U[e] += c.d2c0[d] * s.u[e];
        d2T += c.d2c0[d] * s.Tm;
        Rr -= T(0.5) * (dM[d] + s.u[d] * dRho + s.rho * dU);
#pragma unroll
        for (int e = 0; e < 3; ++e) Rm[e] += c.inv_Re * d2U[e] - T(0.5) * (dF[e] + s.u[d] * dM[e] + s.m[e] * dU);
        Rm[d] += c.inv_3Re * (d2U[d] + dTh);
        RE += c.kappa * d2T - T(0.5) * (dH + s.u[d] * dE + s.E * dU);
    }
    const T Rv[5] = {Rr, Rm[0], Rm[1], Rm[2], RE};
    const T qv[5] = {s.rho, s.m[0], s.m[1], s.m[2], s.E};
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        if (MODE == kModeRHS) {
            out[f * P + id] = Rv[f];
        } else {
            T dn = dt * Rv[f];
            if (MODE != kModeStage1) dn += A * dq[f * P + id];
            if (MODE != kModeStage3) dq[f * P + id] = dn;
            out[f * P + id] = qv[f] + B * dn;
        }
    }
}

}  // namespace sbli
