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
constexpr int kDiagThreads = 256;  // threads of the final reduction
constexpr int kDiagBlocks = 1024;  // fixed grid: deterministic reduction order
constexpr int kDiagZ = 32;         // z-planes per work item of the partial kernel

// Doubles of LDS the block reduction of NT threads needs.
template <int NT>
constexpr int diag_reduce_doubles() { return 2 * kDiagQ * NT + (3 * NT + 1) / 2; }

// Block-level compensated reduction of kDiagQ pairs and 3 counters held per
// thread, in LDS scratch `lds` of diag_reduce_doubles<NT>() doubles; thread 0
// returns the block result.
template <int NT>
__device__ __forceinline__ void block_reduce_diag(CSum (&acc)[kDiagQ], unsigned (&cnt)[3], double* lds) {
    double(*ss)[NT] = reinterpret_cast<double(*)[NT]>(lds);
    double(*sc)[NT] = reinterpret_cast<double(*)[NT]>(lds + kDiagQ * NT);
    unsigned(*sn)[NT] = reinterpret_cast<unsigned(*)[NT]>(lds + 2 * kDiagQ * NT);
    const int t = threadIdx.x;
    for (int d = 0; d < kDiagQ; ++d) { ss[d][t] = acc[d].s; sc[d][t] = acc[d].c; }
    for (int d = 0; d < 3; ++d) sn[d][t] = cnt[d];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
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

// Tile of the partial kernel: 16 x TY columns (TY = 8 for the wide stencils,
// which keeps the LDS rings small enough for four workgroups per CU, so that
// the fixed grid runs in one round).
template <int R>
struct DiagShape {
    static constexpr int TX = 16;
    static constexpr int TY = R <= 3 ? 16 : 8;
    static constexpr int NT = TX * TY;
    static constexpr int MINW = R <= 3 ? 4 : 2;                   // wavefronts per SIMD to allow
    static constexpr int NR = 2 * R + 1;                           // planes of (u0, u1) in the ring
    static constexpr int RING = NR * 2 * TY * TX + (R + 1) * TY * TX;   // and R+1 planes of u2
    static constexpr int HALO = 2 * 2 * TY * R + 2 * 2 * R * TX;   // (u1, u2) x-ring, (u0, u2) y-ring
    static constexpr int LDS = RING + HALO > diag_reduce_doubles<NT>() ? RING + HALO : diag_reduce_doubles<NT>();
};

// Per-block partial sums of the diagnostics.  Every value is converted to
// double before any arithmetic.  Vorticity uses the order-2R central first
// derivative with weights da (a_m / h, double) of u = m / rho, each taken with
// one IEEE division per point.  A block takes work items (a tile of columns and
// a chunk of kDiagZ planes) in a fixed round-robin order and marches each in z:
// (u0, u1) of the tile's columns over the last 2R+1 planes and u2 over the last
// R+1 (only the centre plane's is differentiated) sit in LDS rings, and the
// tangential components of the centre plane's x and y rings are loaded per plane.
// part layout: [block][2*kDiagQ doubles (s, c pairs)] then counters [block][3]
// (as doubles).
template <typename T, int R>
__global__ void __launch_bounds__(DiagShape<R>::NT, DiagShape<R>::MINW) diag_partial_kernel(const T* __restrict__ q, int nx, int ny, int nz,
                                                                        const double* __restrict__ da, double gm1,
                                                                        int symx, int symy, int symz,
                                                                        double* __restrict__ part) {
    using S = DiagShape<R>;
    constexpr int TX = S::TX, TY = S::TY, NT = S::NT, NR = S::NR;
    __shared__ double s_lds[S::LDS];
    double(*s_u)[2][TY][TX] = reinterpret_cast<double(*)[2][TY][TX]>(s_lds);            // [slot][u0,u1][y][x]
    double(*s_w)[TY][TX] = reinterpret_cast<double(*)[TY][TX]>(s_lds + NR * 2 * TY * TX);  // [slot][y][x] of u2
    double(*s_hx)[2][TY][R] = reinterpret_cast<double(*)[2][TY][R]>(s_lds + S::RING);    // [side][u1,u2][y][m]
    double(*s_hy)[2][R][TX] = reinterpret_cast<double(*)[2][R][TX]>(s_lds + S::RING + 4 * TY * R);  // [side][u0,u2][m][x]

    const int64_t P = (int64_t)nx * ny * nz;
    const int64_t plane = (int64_t)nx * ny;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    double w[3][R];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int m = 0; m < R; ++m) w[a][m] = da[a * kMaxR + m];

    CSum acc[kDiagQ];
    for (int d = 0; d < kDiagQ; ++d) acc[d] = CSum{0.0, 0.0};
    unsigned cnt[3] = {0u, 0u, 0u};

    const int tiles_x = (nx + TX - 1) / TX, tiles_y = (ny + TY - 1) / TY;
    const int items = tiles_x * tiles_y * ((nz + kDiagZ - 1) / kDiagZ);
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tile = it % (tiles_x * tiles_y), chunk = it / (tiles_x * tiles_y);
        const int x0 = (tile % tiles_x) * TX, y0 = (tile / tiles_x) * TY;
        const int z0 = chunk * kDiagZ, z1 = min(nz, z0 + kDiagZ);
        unsigned f;
        // the tile's columns as a window of the wrapped (or mirrored) box: a
        // column beyond the box holds the values of the point it folds onto
        const int64_t col = (int64_t)fold_index(y0 + ty, ny, symy, f) * nx + fold_index(x0 + tx, nx, symx, f);
        const bool own = (x0 + tx < nx) && (y0 + ty < ny);
        auto slot = [&](int k) { return (k - z0 + R) % NR; };
        auto wslot = [&](int k) { return (k - z0 + R) % (R + 1); };
        // planes are loaded in increasing order, so a u2 slot that two warm-up
        // planes share ends up holding the later one, the only one differentiated
        auto load_plane = [&](int k) {
            const int64_t id = (int64_t)fold_index(k, nz, symz, f) * plane + col;
            const double rho = (double)q[id];
            s_u[slot(k)][0][ty][tx] = (double)q[P + id] / rho;
            s_u[slot(k)][1][ty][tx] = (double)q[2 * P + id] / rho;
            s_w[wslot(k)][ty][tx] = (double)q[3 * P + id] / rho;
        };
        __syncthreads();   // the previous work item's reads of the ring are done
        for (int k = z0 - R; k < z0 + R; ++k) load_plane(k);
        for (int k = z0; k < z1; ++k) {
            load_plane(k + R);
            // x and y rings of plane k (no corners): the components tangential to each
            const int64_t pz = (int64_t)k * plane;
            for (int h = tid; h < 2 * R * (TX + TY); h += NT) {
                if (h < 2 * R * TY) {
                    const int side = h / (R * TY), r = h % (R * TY), hy = r / R, m = r % R;
                    const int gx = fold_index(side ? x0 + TX + m : x0 - R + m, nx, symx, f);
                    const int64_t id = pz + (int64_t)fold_index(y0 + hy, ny, symy, f) * nx + gx;
                    const double rho = (double)q[id];
                    s_hx[side][0][hy][m] = (double)q[2 * P + id] / rho;
                    s_hx[side][1][hy][m] = (double)q[3 * P + id] / rho;
                } else {
                    const int h2 = h - 2 * R * TY;
                    const int side = h2 / (R * TX), r = h2 % (R * TX), m = r / TX, hx = r % TX;
                    const int gy = fold_index(side ? y0 + TY + m : y0 - R + m, ny, symy, f);
                    const int64_t id = pz + (int64_t)gy * nx + fold_index(x0 + hx, nx, symx, f);
                    const double rho = (double)q[id];
                    s_hy[side][0][m][hx] = (double)q[P + id] / rho;
                    s_hy[side][1][m][hx] = (double)q[3 * P + id] / rho;
                }
            }
            __syncthreads();
            if (own) {
                const int c = slot(k), cw = wslot(k);
                // derivatives of u_b along axis a: dudy, dudz, dvdx, dvdz, dwdx, dwdy.
                // Each component is differentiated across the axes it is tangential
                // to, so on a symmetry axis its mirror image has the same sign.
                double dvdx = 0, dwdx = 0, dudy = 0, dwdy = 0, dudz = 0, dvdz = 0;
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    {
                        const double vp = tx + m < TX ? s_u[c][1][ty][tx + m] : s_hx[1][0][ty][tx + m - TX];
                        const double wp = tx + m < TX ? s_w[cw][ty][tx + m] : s_hx[1][1][ty][tx + m - TX];
                        const double vm = tx - m >= 0 ? s_u[c][1][ty][tx - m] : s_hx[0][0][ty][tx - m + R];
                        const double wm = tx - m >= 0 ? s_w[cw][ty][tx - m] : s_hx[0][1][ty][tx - m + R];
                        dvdx += w[0][m - 1] * (vp - vm);
                        dwdx += w[0][m - 1] * (wp - wm);
                    }
                    {
                        const double up = ty + m < TY ? s_u[c][0][ty + m][tx] : s_hy[1][0][ty + m - TY][tx];
                        const double wp = ty + m < TY ? s_w[cw][ty + m][tx] : s_hy[1][1][ty + m - TY][tx];
                        const double um = ty - m >= 0 ? s_u[c][0][ty - m][tx] : s_hy[0][0][ty - m + R][tx];
                        const double wm = ty - m >= 0 ? s_w[cw][ty - m][tx] : s_hy[0][1][ty - m + R][tx];
                        dudy += w[1][m - 1] * (up - um);
                        dwdy += w[1][m - 1] * (wp - wm);
                    }
                    {
                        const int cp = slot(k + m), cm = slot(k - m);
                        dudz += w[2][m - 1] * (s_u[cp][0][ty][tx] - s_u[cm][0][ty][tx]);
                        dvdz += w[2][m - 1] * (s_u[cp][1][ty][tx] - s_u[cm][1][ty][tx]);
                    }
                }
                const int64_t id = pz + col;
                const double rho = (double)q[id];
                const double m0 = (double)q[P + id], m1 = (double)q[2 * P + id], m2 = (double)q[3 * P + id];
                const double rE = (double)q[4 * P + id];
                const double u0 = s_u[c][0][ty][tx], u1 = s_u[c][1][ty][tx], u2 = s_w[cw][ty][tx];
                const double wx = dwdy - dvdz, wy = dudz - dwdx, wz = dvdx - dudy;
                acc[0] = csum_add(acc[0], 0.5 * rho * (u0 * u0 + u1 * u1 + u2 * u2));
                acc[1] = csum_add(acc[1], 0.5 * rho * (wx * wx + wy * wy + wz * wz));
                const double qf[5] = {rho, m0, m1, m2, rE};
                for (int fi = 0; fi < 5; ++fi) {
                    acc[2 + fi] = csum_add(acc[2 + fi], qf[fi]);
                    cnt[0] += isfinite(qf[fi]) ? 0u : 1u;
                }
                const double p = gm1 * (rE - 0.5 * (m0 * u0 + m1 * u1 + m2 * u2));
                cnt[1] += (rho > 0.0) ? 0u : 1u;
                cnt[2] += (p > 0.0) ? 0u : 1u;
            }
            __syncthreads();   // plane k's ring slot and rings are read before they are replaced
        }
    }
    block_reduce_diag<NT>(acc, cnt, s_lds);
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
    __shared__ double s_lds[diag_reduce_doubles<kDiagThreads>()];
    CSum acc[kDiagQ];
    for (int d = 0; d < kDiagQ; ++d) acc[d] = CSum{0.0, 0.0};
    unsigned cnt[3] = {0u, 0u, 0u};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const double* o = part + (int64_t)b * (2 * kDiagQ + 3);
        for (int d = 0; d < kDiagQ; ++d) acc[d] = csum_merge(acc[d], CSum{o[2 * d], o[2 * d + 1]});
        for (int d = 0; d < 3; ++d) cnt[d] += (unsigned)o[2 * kDiagQ + d];
    }
    block_reduce_diag<kDiagThreads>(acc, cnt, s_lds);
    if (threadIdx.x == 0) {
        for (int d = 0; d < kDiagQ; ++d) out[d] = (acc[d].s + acc[d].c) * inv_P;
        for (int d = 0; d < 3; ++d) out[kDiagQ + d] = (double)cnt[d];
    }
}

}  // namespace sbli
