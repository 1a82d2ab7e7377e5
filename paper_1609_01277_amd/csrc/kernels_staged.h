// Staged form of the residual and RK3 stage: three point-parallel launches with
// the intermediate fields in HBM.  It serves every order 2..12 (the fused stage
// kernel's register window and LDS planes do not fit beyond order 8) and is a
// launch variant of the lower orders as well, where it reproduces the fused
// kernel bit for bit: both compute the same per-point arithmetic in the same
// order (make_pf, the gradient sums, DirSums::add / finish, the 2N update).
//
//   1. staged_point_kernel:  w = (u_0, u_1, u_2, p, T) of every point;
//   2. staged_nested_kernel: nf = (V_0, V_1, V_2, theta - g_00, theta - g_11,
//      theta - g_22) with g_ij = D_j u_i, V_j = u_i tau_ij (paper Sec.
//      "Expanding": the inner derivative of a nested term is taken first);
//   3. staged_stage_kernel:  the residual (paper eqs. of mass, momentum and
//      energy in the skew-symmetric form) from q, w and nf at the 2R
//      neighbours along each axis, then the 2N Runge-Kutta update.
//
// On a symmetry axis a neighbour beyond the boundary is the mirror image of an
// inside point; the components normal to that boundary of the momentum, the
// velocity and V (an odd field) change sign, exactly.
#pragma once

#include "kernels_stage_fused.h"

namespace sbli {

constexpr int kStagedThreads = 256;

// Linear index of the neighbour m points away along an axis (coordinate c,
// stride `stride`, n points, sym = mirrored ends); `flip` gets the sign mask.
__device__ __forceinline__ int64_t staged_nb(int64_t id, int c, int m, int n, int64_t stride, int sym,
                                             unsigned& flip) {
    const int cc = map_index(c + m, n, sym, flip);
    return id + (int64_t)(cc - c) * stride;
}

template <typename T>
__global__ void __launch_bounds__(kStagedThreads)
    staged_point_kernel(const T* __restrict__ q, T* __restrict__ w, int64_t P, T gm1, T gM2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < P; id += stride) {
        const PF<T> f = make_pf<T>(q[id], q[P + id], q[2 * P + id], q[3 * P + id], q[4 * P + id], gm1, gM2);
        w[id] = f.u0;
        w[P + id] = f.u1;
        w[2 * P + id] = f.u2;
        w[3 * P + id] = f.p;
        w[4 * P + id] = f.Tm;
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(kStagedThreads)
    staged_nested_kernel(const T* __restrict__ w, T* __restrict__ nf, const BoxConst<T> c) {
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int64_t P = c.P, sy = nx, sz = (int64_t)nx * ny;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < P; id += stride) {
        const int i = (int)(id % nx);
        const int64_t t = id / nx;
        const int j = (int)(t % ny);
        const int k = (int)(t / ny);
        T g[3][3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            T sx = 0, syy = 0, szz = 0;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                unsigned fp, fm;
                int64_t ip = staged_nb(id, i, m, nx, 1, c.sym[0], fp), im = staged_nb(id, i, -m, nx, 1, c.sym[0], fm);
                T up = w[b * P + ip], um = w[b * P + im];
                if (b == 0) { up = flip_sign(up, fp); um = flip_sign(um, fm); }
                sx = fmaT(c.da[0][m - 1], up - um, sx);
                ip = staged_nb(id, j, m, ny, sy, c.sym[1], fp);
                im = staged_nb(id, j, -m, ny, sy, c.sym[1], fm);
                up = w[b * P + ip];
                um = w[b * P + im];
                if (b == 1) { up = flip_sign(up, fp); um = flip_sign(um, fm); }
                syy = fmaT(c.da[1][m - 1], up - um, syy);
                ip = staged_nb(id, k, m, nz, sz, c.sym[2], fp);
                im = staged_nb(id, k, -m, nz, sz, c.sym[2], fm);
                up = w[b * P + ip];
                um = w[b * P + im];
                if (b == 2) { up = flip_sign(up, fp); um = flip_sign(um, fm); }
                szz = fmaT(c.da[2][m - 1], up - um, szz);
            }
            g[b][0] = sx;
            g[b][1] = syy;
            g[b][2] = szz;
        }
        const T uc[3] = {w[id], w[P + id], w[2 * P + id]};
        const T theta = g[0][0] + g[1][1] + g[2][2];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            T v = 0;
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) {
                T tau = c.inv_Re * (g[ii][jj] + g[jj][ii]);
                if (ii == jj) tau = fmaT(-c.inv_Re23, theta, tau);
                v = fmaT(uc[ii], tau, v);
            }
            nf[jj * P + id] = v;
            nf[(3 + jj) * P + id] = theta - g[jj][jj];
        }
    }
}

template <typename T, int R, int MODE>
__global__ void __launch_bounds__(kStagedThreads)
    staged_stage_kernel(const T* __restrict__ q, const T* __restrict__ w, const T* __restrict__ nf,
                        T* __restrict__ dq, T* __restrict__ out, const BoxConst<T> c, T dt, T A, T B,
                        const T* __restrict__ clos, const int* __restrict__ cflag) {
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int64_t P = c.P, sy = nx, sz = (int64_t)nx * ny;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // point fields of point ix with the component along axis d sign-masked
    auto point = [&](int64_t ix, int d, unsigned f) {
        PF<T> p;
        p.rho = q[ix];
        p.m0 = q[P + ix];
        p.m1 = q[2 * P + ix];
        p.m2 = q[3 * P + ix];
        p.E = q[4 * P + ix];
        p.u0 = w[ix];
        p.u1 = w[P + ix];
        p.u2 = w[2 * P + ix];
        p.p = w[3 * P + ix];
        p.Tm = w[4 * P + ix];
        if (d == 0) { p.m0 = flip_sign(p.m0, f); p.u0 = flip_sign(p.u0, f); }
        if (d == 1) { p.m1 = flip_sign(p.m1, f); p.u1 = flip_sign(p.u1, f); }
        if (d == 2) { p.m2 = flip_sign(p.m2, f); p.u2 = flip_sign(p.u2, f); }
        return p;
    };
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < P; id += stride) {
        const int coord[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((int64_t)nx * ny))};
        const int64_t stv[3] = {1, sy, sz};
        const PF<T> s = point(id, -1, 0u);
        T Rr = 0, R0 = 0, R1 = 0, R2 = 0, RE = 0;
        static_for<3>([&](auto dd) {
            constexpr int d = decltype(dd)::value;
            DirSums<T> ds;
            ds.zero();
            // not unrolled: unrolled, the compiler requests every neighbour of the
            // axis at once and spills the registers that needs
#pragma unroll 1
            for (int m = 1; m <= R; ++m) {
                unsigned fa, fb;
                const int64_t ia = staged_nb(id, coord[d], m, c.n[d], stv[d], c.sym[d], fa);
                const int64_t ib = staged_nb(id, coord[d], -m, c.n[d], stv[d], c.sym[d], fb);
                ds.template add<d>(point(ia, d, fa), flip_sign(nf[d * P + ia], fa), nf[(3 + d) * P + ia],
                                   point(ib, d, fb), flip_sign(nf[d * P + ib], fb), nf[(3 + d) * P + ib],
                                   c.da[d][m - 1], c.d2c[d][m - 1]);
            }
            ds.template finish<d>(s, c.d2c0[d], c, Rr, R0, R1, R2, RE);
        });
        T Rv[5] = {Rr, R0, R1, R2, RE};
        if (clos != nullptr && cflag[0] != 0) {
#pragma unroll
            for (int f = 0; f < 5; ++f) Rv[f] += clos[f * P + id];
        }
        const T qv[5] = {s.rho, s.m0, s.m1, s.m2, s.E};
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            if (MODE == kModeRHS) {
                out[f * P + id] = Rv[f];
            } else {
                T dn = dt * Rv[f];
                if (MODE != kModeStage1) dn = fmaT(A, dq[f * P + id], dn);
                if (MODE != kModeStage3) dq[f * P + id] = dn;
                out[f * P + id] = fmaT(B, dn, qv[f]);
            }
        }
    }
}

}  // namespace sbli
