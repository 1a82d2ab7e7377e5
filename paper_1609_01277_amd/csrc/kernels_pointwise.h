// Point-per-thread kernels: Taylor-Green initial state and the diagnostics
// reduction (kinetic energy, enstrophy, conservation sums).
#pragma once

#include "sbli_common.h"

namespace sbli {

// Taylor-Green initial condition (paper Sec. "3D Taylor-Green vortex"), L = 1,
// rho = 1, evaluated in double and stored in T.
template <typename T>
__global__ void __launch_bounds__(256) tgv_init_kernel(T* __restrict__ q, int nx, int ny, int nz,
                                                        double hx, double hy, double hz,
                                                        double px, double py, double pz,
                                                        double gamma, double mach) {
    const int64_t P = (int64_t)nx * ny * nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= P) return;
    const int i = (int)(id % nx);
    const int64_t t = id / nx;
    const int j = (int)(t % ny);
    const int k = (int)(t / ny);
    const double x = i * hx + px, y = j * hy + py, z = k * hz + pz;
    double sx, cx, sy, cy, sz, cz;
    sincos(x, &sx, &cx);
    sincos(y, &sy, &cy);
    sincos(z, &sz, &cz);
    const double u = sx * cy * cz;
    const double v = -cx * sy * cz;
    const double rho = 1.0;
    const double p = 1.0 / (gamma * mach * mach) + (cos(2.0 * x) + cos(2.0 * y)) * (cos(2.0 * z) + 2.0) / 16.0;
    q[id] = (T)rho;
    q[P + id] = (T)(rho * u);
    q[2 * P + id] = (T)(rho * v);
    q[3 * P + id] = (T)0.0;
    q[4 * P + id] = (T)(p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v));
}

// Compensated (sum, error) pair; combining two pairs keeps the rounding error of
// the addition (Knuth TwoSum), so a tree of combinations is as accurate as a
// sequential Neumaier sum.
struct CSum {
    double s, c;
};

__device__ __forceinline__ CSum csum_add(CSum a, double x) {
    const double t = a.s + x;
    const double bp = t - a.s;
    const double e = (a.s - (t - bp)) + (x - bp);
    return CSum{t, a.c + e};
}

__device__ __forceinline__ CSum csum_merge(CSum a, CSum b) {
    CSum r = csum_add(a, b.s);
    r.c += b.c;
    return r;
}

constexpr int kDiagQ = 7;          // E_k, enstrophy, 5 conservation sums
constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 1024;  // fixed grid: deterministic reduction order

// Block-level compensated reduction of kDiagQ pairs and 3 counters held per
// thread; thread 0 returns the block result.
__device__ __forceinline__ void block_reduce_diag(CSum (&acc)[kDiagQ], unsigned (&cnt)[3]) {
    __shared__ double ss[kDiagQ][kDiagThreads];
    __shared__ double sc[kDiagQ][kDiagThreads];
    __shared__ unsigned sn[3][kDiagThreads];
    const int t = threadIdx.x;
    for (int d = 0; d < kDiagQ; ++d) { ss[d][t] = acc[d].s; sc[d][t] = acc[d].c; }
    for (int d = 0; d < 3; ++d) sn[d][t] = cnt[d];
    __syncthreads();
    for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            for (int d = 0; d < kDiagQ; ++d) {
                CSum r = csum_merge(CSum{ss[d][t], sc[d][t]}, CSum{ss[d][t + w], sc[d][t + w]});
                ss[d][t] = r.s;
                sc[d][t] = r.c;
            }
            for (int d = 0; d < 3; ++d) sn[d][t] += sn[d][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int d = 0; d < kDiagQ; ++d) acc[d] = CSum{ss[d][0], sc[d][0]};
        for (int d = 0; d < 3; ++d) cnt[d] = sn[d][0];
    }
}

// Per-block partial sums of the diagnostics.  Every value is converted to
// double before any arithmetic.  Vorticity uses the order-2R central first
// derivative with weights da (a_m / h, double).  part layout:
// [block][2*kDiagQ doubles (s, c pairs)] then counters [block][3] (as doubles).
template <typename T, int R>
__global__ void __launch_bounds__(kDiagThreads) diag_partial_kernel(const T* __restrict__ q, int nx, int ny, int nz,
                                                                    const double* __restrict__ da, double gm1,
                                                                    int symx, int symy, int symz,
                                                                    double* __restrict__ part) {
    const int64_t P = (int64_t)nx * ny * nz;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    CSum acc[kDiagQ];
    for (int d = 0; d < kDiagQ; ++d) acc[d] = CSum{0.0, 0.0};
    unsigned cnt[3] = {0u, 0u, 0u};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < P; id += stride) {
        const int i = (int)(id % nx);
        const int64_t t = id / nx;
        const int j = (int)(t % ny);
        const int k = (int)(t / ny);
        const double rho = (double)q[id];
        const double m0 = (double)q[P + id], m1 = (double)q[2 * P + id], m2 = (double)q[3 * P + id];
        const double rE = (double)q[4 * P + id];
        const double u0 = m0 / rho, u1 = m1 / rho, u2 = m2 / rho;
        // derivatives of u_b along axis a: dudy, dudz, dvdx, dvdz, dwdx, dwdy.  Each
        // component is differentiated across the axes it is tangential to, so on
        // a symmetry axis its mirror image has the same sign.
        double dvdx = 0, dwdx = 0, dudy = 0, dwdy = 0, dudz = 0, dvdz = 0;
#pragma unroll
        for (int m = 1; m <= R; ++m) {
            {
                const int64_t ip = shifted(id, i, m, nx, 1, symx), im = shifted(id, i, -m, nx, 1, symx);
                const double rp = (double)q[ip], rm = (double)q[im];
                const double w = da[0 * kMaxR + m - 1];
                dvdx += w * ((double)q[2 * P + ip] / rp - (double)q[2 * P + im] / rm);
                dwdx += w * ((double)q[3 * P + ip] / rp - (double)q[3 * P + im] / rm);
            }
            {
                const int64_t ip = shifted(id, j, m, ny, sy, symy), im = shifted(id, j, -m, ny, sy, symy);
                const double rp = (double)q[ip], rm = (double)q[im];
                const double w = da[1 * kMaxR + m - 1];
                dudy += w * ((double)q[P + ip] / rp - (double)q[P + im] / rm);
                dwdy += w * ((double)q[3 * P + ip] / rp - (double)q[3 * P + im] / rm);
            }
            {
                const int64_t ip = shifted(id, k, m, nz, sz, symz), im = shifted(id, k, -m, nz, sz, symz);
                const double rp = (double)q[ip], rm = (double)q[im];
                const double w = da[2 * kMaxR + m - 1];
                dudz += w * ((double)q[P + ip] / rp - (double)q[P + im] / rm);
                dvdz += w * ((double)q[2 * P + ip] / rp - (double)q[2 * P + im] / rm);
            }
        }
        const double wx = dwdy - dvdz, wy = dudz - dwdx, wz = dvdx - dudy;
        acc[0] = csum_add(acc[0], 0.5 * rho * (u0 * u0 + u1 * u1 + u2 * u2));
        acc[1] = csum_add(acc[1], 0.5 * rho * (wx * wx + wy * wy + wz * wz));
        const double qf[5] = {rho, m0, m1, m2, rE};
        for (int f = 0; f < 5; ++f) {
            acc[2 + f] = csum_add(acc[2 + f], qf[f]);
            cnt[0] += isfinite(qf[f]) ? 0u : 1u;
        }
        const double p = gm1 * (rE - 0.5 * (m0 * u0 + m1 * u1 + m2 * u2));
        cnt[1] += (rho > 0.0) ? 0u : 1u;
        cnt[2] += (p > 0.0) ? 0u : 1u;
    }
    block_reduce_diag(acc, cnt);
    if (threadIdx.x == 0) {
        double* o = part + (int64_t)blockIdx.x * (2 * kDiagQ + 3);
        for (int d = 0; d < kDiagQ; ++d) { o[2 * d] = acc[d].s; o[2 * d + 1] = acc[d].c; }
        for (int d = 0; d < 3; ++d) o[2 * kDiagQ + d] = (double)cnt[d];
    }
}

// Single-block reduction of the per-block partials, in a fixed order.
// out[0..6] = averages (sum / P), out[7..9] = counters.
__global__ void __launch_bounds__(kDiagThreads) diag_final_kernel(const double* __restrict__ part, int nblocks,
                                                                  double inv_P, double* __restrict__ out) {
    CSum acc[kDiagQ];
    for (int d = 0; d < kDiagQ; ++d) acc[d] = CSum{0.0, 0.0};
    unsigned cnt[3] = {0u, 0u, 0u};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double* o = part + (int64_t)b * (2 * kDiagQ + 3);
        for (int d = 0; d < kDiagQ; ++d) acc[d] = csum_merge(acc[d], CSum{o[2 * d], o[2 * d + 1]});
        for (int d = 0; d < 3; ++d) cnt[d] += (unsigned)o[2 * kDiagQ + d];
    }
    block_reduce_diag(acc, cnt);
    if (threadIdx.x == 0) {
        for (int d = 0; d < kDiagQ; ++d) out[d] = (acc[d].s + acc[d].c) * inv_P;
        for (int d = 0; d < 3; ++d) out[kDiagQ + d] = (double)cnt[d];
    }
}

}  // namespace sbli
