// Staged form of the residual and RK3 stage: two launches, one thread per
// point, with the nested fields in HBM between them.  It serves every order
// 2..12 (the fused stage kernel's register window and LDS planes do not fit
// beyond order 8) and is a launch variant of the lower orders as well, where it
// reproduces the fused kernel bit for bit: both compute the same per-point
// arithmetic in the same order (make_pf, the gradient sums, DirSums::add /
// finish, the 2N update).  The point fields (u_i, p, T) are recomputed by
// make_pf from q wherever a point is read; the same function of the same inputs,
// they are the values the fused kernel keeps in its window.
//
//   1. staged_nested_zring_kernel: nf = (V_0, V_1, V_2, theta - g_00,
//      theta - g_11, theta - g_22) with g_ij = D_j u_i, V_j = u_i tau_ij (paper
//      Sec. "Expanding": the inner derivative of a nested term is taken first);
//   2. staged_tiled_kernel:  the residual (paper eqs. of mass, momentum and
//      energy in the skew-symmetric form) from q and nf at the 2R neighbours
//      along each axis, then the 2N Runge-Kutta update.
//
// On a symmetry axis a neighbour beyond the boundary is the mirror image of an
// inside point; the components normal to that boundary of the momentum, the
// velocity and V (an odd field) change sign, exactly.  Negating a momentum
// component before make_pf negates the matching velocity and leaves p and T
// unchanged, bit for bit, so the sign may be applied before or after.
#pragma once

#include "kernels_stage_fused.h"

namespace sbli {

// Both steps run in tiles: a workgroup owns a square tile of (x, y) columns
// (kStagedTile wide in the residual step; twice that in the nested-field step
// where registers and LDS allow, see staged.hip) and a run of zchunk z-planes (the
// residual step runs one plane per workgroup, the nested-field step runs of
// kNestedRun; see staged_unit).  Per
// plane it stages what the x/y stencils read into LDS, so every element is
// loaded once instead of once per neighbour that needs it.  The z neighbours of
// the thread's own column come from memory in the residual step and from a
// register ring in the nested-field step.
//
// The residual step stages one strip at a time: the tile with its x arms (TS rows
// of TS + 2R points) for the x sums, then the tile with its y arms (TS + 2R rows of
// TS points) in the same LDS for the y sums.  Each thread keeps its own point in
// registers and writes it into both strips; only the arms are loaded by the
// workgroup.  A strip holds the ten point fields and the nested pair of its axis,
// which keeps a workgroup's LDS small enough that registers, not LDS, bound the
// number of workgroups per CU up to order 12.
constexpr int kStagedTile = 16;
// Planes per run of the z-marching nested-field step (2R planes of the own
// column are loaded ahead of each run).  Runs of 32 and 128 measure the same at
// 512^3, orders 8 and 12.
constexpr int kNestedRun = 64;
constexpr int kStagedFields = 12;   // rho, rho u_i, rho E, u_i, p, T, then V_d, theta - g_dd of the axis d

// The unit of work of a tiled launch is (tile, run of zc planes).  Units are
// numbered by pairs of x-adjacent tiles, plane run by plane run within a pair
// (a last unpaired tile comes alone).  Workgroups go to the 8 XCDs round-robin
// by id, and XCD k takes the k-th contiguous eighth of the units in order, so the
// workgroups resident on one XCD hold neighbouring planes of the same two tiles
// at a time: the z neighbours they read (2R planes on either side) and the x arms
// the pair shares are then found in that XCD's L2, instead of each workgroup
// streaming a window of its own through it.  The grid has 8 * ceil(units / 8)
// workgroups; the few beyond the last unit exit.
constexpr int kStagedXcds = 8;
constexpr int kStagedPair = 2;

__device__ __forceinline__ bool staged_unit(int ntiles, int nchunks, int& tile, int& chunk) {
    const int64_t units = (int64_t)ntiles * nchunks;
    const int64_t per = (units + kStagedXcds - 1) / kStagedXcds;
    const int64_t u = (int64_t)(blockIdx.x % kStagedXcds) * per + blockIdx.x / kStagedXcds;
    if (u >= units) return false;
    constexpr int G = kStagedPair;
    const int64_t paired = (int64_t)(ntiles / G) * G * nchunks;
    if (u < paired) {
        const int64_t g = u / (G * nchunks), r = u % (G * nchunks);
        chunk = (int)(r / G);
        tile = (int)(g * G + r % G);
    } else {   // the last ntiles % G tiles, one after the other
        const int rest = ntiles % G;
        const int64_t r = u - paired;
        chunk = (int)(r / rest);
        tile = (ntiles / G) * G + (int)(r % rest);
    }
    return true;
}

template <typename T, int R, int MODE>
__global__ void __launch_bounds__(kStagedTile * kStagedTile)
    staged_tiled_kernel(const T* __restrict__ q, const T* __restrict__ nf,
                        T* __restrict__ dq, T* __restrict__ out, const BoxConst<T> c, T dt, T A, T B,
                        const T* __restrict__ clos, const int* __restrict__ cflag, int tiles_x, int tiles_y,
                        int zchunk) {
    constexpr int TS = kStagedTile, SW = TS + 2 * R, NT = TS * TS, NA = 2 * R * TS;
    __shared__ T sb[kStagedFields][TS * SW];
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int64_t P = c.P, plane = (int64_t)nx * ny;
    int tile, chunk;
    if (!staged_unit(tiles_x * tiles_y, (nz + zchunk - 1) / zchunk, tile, chunk)) return;
    const int z0 = chunk * zchunk;
    const int z1 = min(z0 + zchunk, nz);
    const int x0 = (tile % tiles_x) * TS, y0 = (tile / tiles_x) * TS;
    const int tid = threadIdx.x, cx = tid % TS, cy = tid / TS;
    const bool store = x0 + cx < nx && y0 + cy < ny;
    // own column, folded for lanes of a ragged tile: their results are not stored,
    // but their (mirrored) points are the neighbours of the last columns inside
    unsigned fxo, fyo;
    const int64_t col = (int64_t)fold_index(y0 + cy, ny, c.sym[1], fyo) * nx + fold_index(x0 + cx, nx, c.sym[0], fxo);
    auto point_at = [&](int64_t ix) {
        return make_pf<T>(q[ix], q[P + ix], q[2 * P + ix], q[3 * P + ix], q[4 * P + ix], c.gm1, c.gM2);
    };
    auto lds_point = [&](int i) {
        PF<T> p;
        p.rho = sb[0][i];
        p.m0 = sb[1][i];
        p.m1 = sb[2][i];
        p.m2 = sb[3][i];
        p.E = sb[4][i];
        p.u0 = sb[5][i];
        p.u1 = sb[6][i];
        p.u2 = sb[7][i];
        p.p = sb[8][i];
        p.Tm = sb[9][i];
        return p;
    };
    // a point mirrored across x (fx) and/or y (fy), and the nested pair of the strip
    auto put = [&](int i, const PF<T>& p, unsigned fx, unsigned fy, T v, T th) {
        sb[0][i] = p.rho;
        sb[1][i] = flip_sign(p.m0, fx);
        sb[2][i] = flip_sign(p.m1, fy);
        sb[3][i] = p.m2;
        sb[4][i] = p.E;
        sb[5][i] = flip_sign(p.u0, fx);
        sb[6][i] = flip_sign(p.u1, fy);
        sb[7][i] = p.u2;
        sb[8][i] = p.p;
        sb[9][i] = p.Tm;
        sb[10][i] = v;
        sb[11][i] = th;
    };
    for (int z = z0; z < z1; ++z) {
        const int64_t pz = (int64_t)z * plane, id = pz + col;
        const PF<T> s = point_at(id);
        T Rr = 0, R0 = 0, R1 = 0, R2 = 0, RE = 0;
        __syncthreads();   // the previous plane's y-strip reads are done
        put(cy * SW + R + cx, s, fxo, fyo, flip_sign(nf[id], fxo), nf[3 * P + id]);   // V_x: odd under an x mirror
        for (int e = tid; e < NA; e += NT) {
            const int side = e / (R * TS), r = e % (R * TS);
            const int ly = r / R, lx = side ? R + TS + r % R : r % R;
            unsigned fx, fy;
            const int64_t ix = pz + (int64_t)fold_index(y0 + ly, ny, c.sym[1], fy) * nx +
                               fold_index(x0 - R + lx, nx, c.sym[0], fx);
            put(ly * SW + lx, point_at(ix), fx, fy, flip_sign(nf[ix], fx), nf[3 * P + ix]);
        }
        __syncthreads();
        {
            const int i = cy * SW + R + cx;
            DirSums<T> ds;
            ds.zero();
#pragma unroll 1
            for (int m = 1; m <= R; ++m)
                ds.template add<0>(lds_point(i + m), sb[10][i + m], sb[11][i + m], lds_point(i - m), sb[10][i - m],
                                   sb[11][i - m], c.da[0][m - 1], c.d2c[0][m - 1]);
            ds.template finish<0>(s, c.d2c0[0], c, Rr, R0, R1, R2, RE);
        }
        __syncthreads();   // the x-strip reads are done
        put((R + cy) * TS + cx, s, fxo, fyo, flip_sign(nf[P + id], fyo), nf[4 * P + id]);   // V_y: odd under a y mirror
        for (int e = tid; e < NA; e += NT) {
            const int side = e / (R * TS), r = e % (R * TS);
            const int lx = r % TS, ly = side ? R + TS + r / TS : r / TS;
            unsigned fx, fy;
            const int64_t ix = pz + (int64_t)fold_index(y0 - R + ly, ny, c.sym[1], fy) * nx +
                               fold_index(x0 + lx, nx, c.sym[0], fx);
            put(ly * TS + lx, point_at(ix), fx, fy, flip_sign(nf[P + ix], fy), nf[4 * P + ix]);
        }
        __syncthreads();
        {
            const int i = (R + cy) * TS + cx;
            DirSums<T> ds;
            ds.zero();
#pragma unroll 1
            for (int m = 1; m <= R; ++m)
                ds.template add<1>(lds_point(i + m * TS), sb[10][i + m * TS], sb[11][i + m * TS], lds_point(i - m * TS),
                                   sb[10][i - m * TS], sb[11][i - m * TS], c.da[1][m - 1], c.d2c[1][m - 1]);
            ds.template finish<1>(s, c.d2c0[1], c, Rr, R0, R1, R2, RE);
        }
        {
            DirSums<T> ds;
            ds.zero();
#pragma unroll 1
            for (int m = 1; m <= R; ++m) {
                unsigned fa, fb;
                const int64_t ia = (int64_t)map_index(z + m, nz, c.sym[2], fa) * plane + col;
                const int64_t ib = (int64_t)map_index(z - m, nz, c.sym[2], fb) * plane + col;
                PF<T> a = point_at(ia), b = point_at(ib);
                a.m2 = flip_sign(a.m2, fa);
                a.u2 = flip_sign(a.u2, fa);
                b.m2 = flip_sign(b.m2, fb);
                b.u2 = flip_sign(b.u2, fb);
                ds.template add<2>(a, flip_sign(nf[2 * P + ia], fa), nf[5 * P + ia], b, flip_sign(nf[2 * P + ib], fb),
                                   nf[5 * P + ib], c.da[2][m - 1], c.d2c[2][m - 1]);
            }
            ds.template finish<2>(s, c.d2c0[2], c, Rr, R0, R1, R2, RE);
        }
        if (store) {
            // dq and the new state are streamed (nothing in this launch reads them
            // again), which leaves L2 to the z neighbours and arms of the tiles
            T Rv[5] = {Rr, R0, R1, R2, RE};
            if (clos != nullptr && cflag[0] != 0) {
#pragma unroll
                for (int f = 0; f < 5; ++f) Rv[f] += clos[f * P + id];
            }
            const T qv[5] = {s.rho, s.m0, s.m1, s.m2, s.E};
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                if (MODE == kModeRHS) {
                    __builtin_nontemporal_store(Rv[f], &out[f * P + id]);
                } else {
                    T dn = dt * Rv[f];
                    if (MODE != kModeStage1) dn = fmaT(A, __builtin_nontemporal_load(&dq[f * P + id]), dn);
                    if (MODE != kModeStage3) __builtin_nontemporal_store(dn, &dq[f * P + id]);
                    __builtin_nontemporal_store(fmaT(B, dn, qv[f]), &out[f * P + id]);
                }
            }
        }
    }
}

// The nested-field step marching in z.  A workgroup owns a tile and a run of
// zchunk planes, and each thread keeps the velocity of its own column over the
// planes z-R..z+R in a register ring (2R+1 planes, rotated by unrolling the plane
// loop 2R+1 times, so every ring index is a compile-time constant).  Per plane
// only the x and y arms of the tile are loaded (one plane ahead, into
// registers); the tile's own points are written into LDS from the ring.  Each
// velocity is formed once per point and plane, as fast_recip(rho) * rho u_i (the
// values the fused kernel's gradient step reads), and the sums over m run in
// ascending order per component and axis, as there.  LDS is double-buffered:
// one barrier per plane.
template <typename T, int R, int TS>
__global__ void __launch_bounds__(TS * TS)
    staged_nested_zring_kernel(const T* __restrict__ q, T* __restrict__ nf, const BoxConst<T> c, int tiles_x,
                               int tiles_y, int zchunk) {
    constexpr int BW = TS + 2 * R, NT = TS * TS, W = 2 * R + 1;
    constexpr int NARM = 4 * R * TS;                  // arm points of a plane (no corners)
    constexpr int APT = (NARM + NT - 1) / NT;         // arm points per thread
    __shared__ T su[2][3][BW][BW];
    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int64_t P = c.P, plane = (int64_t)nx * ny;
    int tile, chunk;
    if (!staged_unit(tiles_x * tiles_y, (nz + zchunk - 1) / zchunk, tile, chunk)) return;
    const int z0 = chunk * zchunk;
    const int run = min(zchunk, nz - z0);
    const int x0 = (tile % tiles_x) * TS, y0 = (tile / tiles_x) * TS;
    const int tid = threadIdx.x, cx = tid % TS, cy = tid / TS;
    const bool store = x0 + cx < nx && y0 + cy < ny;
    unsigned fxo, fyo;
    const int64_t col = (int64_t)fold_index(y0 + cy, ny, c.sym[1], fyo) * nx + fold_index(x0 + cx, nx, c.sym[0], fxo);
    // this thread's arm points: LDS position and column (with its mirror flags)
    int aoff[APT];
    int64_t acol[APT];
    unsigned afx[APT] = {}, afy[APT] = {};
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        const int a = tid + k * NT;
        int lx = 0, ly = 0;
        if (a < NARM) {
            const int side = a / (R * TS), r = a % (R * TS);
            if (side < 2) {
                ly = R + r / R;
                lx = (side == 0 ? 0 : R + TS) + r % R;
            } else {
                lx = R + r % TS;
                ly = (side == 2 ? 0 : R + TS) + r / TS;
            }
        }
        // a thread without this arm point loads its own column instead (unused), so
        // that every wavefront issues the same loads
        aoff[k] = a < NARM ? ly * BW + lx : -1;
        acol[k] = a < NARM ? (int64_t)fold_index(y0 - R + ly, ny, c.sym[1], afy[k]) * nx +
                                 fold_index(x0 - R + lx, nx, c.sym[0], afx[k])
                           : col;
    }
    // velocity of the own column at plane z (mirrored in z when z lies outside)
    auto own_u = [&](int z, T (&u)[3]) {
        unsigned fz;
        const int64_t id = (int64_t)map_index(z, nz, c.sym[2], fz) * plane + col;
        const T rr = fast_recip(q[id]);
        u[0] = q[P + id] * rr;
        u[1] = q[2 * P + id] * rr;
        u[2] = flip_sign(q[3 * P + id] * rr, fz);
    };
    T ring[W][3];
#pragma unroll
    for (int k = 0; k < W; ++k) ring[k][0] = ring[k][1] = ring[k][2] = 0;
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) own_u(z0 - R + k, ring[k]);
    // requested one plane ahead: the own column's entering plane (rho, rho u_i) and
    // the arms of the next centre plane
    T pe[4], pa[APT][4];
    auto issue = [&](int it) {
        unsigned fz;
        const int64_t id = (int64_t)map_index(z0 + it + R, nz, c.sym[2], fz) * plane + col;
        pe[0] = q[id];
        pe[1] = q[P + id];
        pe[2] = q[2 * P + id];
        pe[3] = q[3 * P + id];
        const int64_t pz = (int64_t)(z0 + it) * plane;
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            const int64_t ix = pz + acol[k];
            pa[k][0] = q[ix];
            pa[k][1] = q[P + ix];
            pa[k][2] = q[2 * P + ix];
            pa[k][3] = q[3 * P + ix];
        }
    };
    issue(0);
    auto body = [&](auto ph, const int it) {
        constexpr int PH = decltype(ph)::value;
        auto slot = [](int k) { return (k + PH) % W; };
        const int z = z0 + it;
        const int b = it & 1;
        // the entering plane z + R joins the ring; plane z's arms and tile go to LDS
        {
            unsigned fz;
            map_index(z + R, nz, c.sym[2], fz);
            const T rr = fast_recip(pe[0]);
            ring[slot(2 * R)][0] = pe[1] * rr;
            ring[slot(2 * R)][1] = pe[2] * rr;
            ring[slot(2 * R)][2] = flip_sign(pe[3] * rr, fz);
        }
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (aoff[k] >= 0) {
                const T rr = fast_recip(pa[k][0]);
                T* s0 = &su[b][0][0][0];
                s0[aoff[k]] = flip_sign(pa[k][1] * rr, afx[k]);
                s0[BW * BW + aoff[k]] = flip_sign(pa[k][2] * rr, afy[k]);
                s0[2 * BW * BW + aoff[k]] = pa[k][3] * rr;
            }
        }
        const T (&uc)[3] = ring[slot(R)];
        su[b][0][R + cy][R + cx] = flip_sign(uc[0], fxo);
        su[b][1][R + cy][R + cx] = flip_sign(uc[1], fyo);
        su[b][2][R + cy][R + cx] = uc[2];
        if (it + 1 < run) issue(it + 1);
        __syncthreads();
        const int ly = R + cy, lx = R + cx;
        T g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
        for (int m = 1; m <= R; ++m) {
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                g[bb][0] = fmaT(c.da[0][m - 1], su[b][bb][ly][lx + m] - su[b][bb][ly][lx - m], g[bb][0]);
                g[bb][1] = fmaT(c.da[1][m - 1], su[b][bb][ly + m][lx] - su[b][bb][ly - m][lx], g[bb][1]);
                g[bb][2] = fmaT(c.da[2][m - 1], ring[slot(R + m)][bb] - ring[slot(R - m)][bb], g[bb][2]);
            }
        }
        if (store) {
            const int64_t id = (int64_t)z * plane + col;
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
                __builtin_nontemporal_store(v, &nf[jj * P + id]);
                __builtin_nontemporal_store(theta - g[jj][jj], &nf[(3 + jj) * P + id]);
            }
        } else {
            // as many (dropped) stores, so that waiting for the next plane's loads
            // never has to cover this plane's stores
            dropped_stores<6>(nf);
        }
    };
    for (int it0 = 0; it0 < run; it0 += W) {
        static_for<W>([&](auto ph) {
            const int it = it0 + decltype(ph)::value;
            if (it < run) body(ph, it);
        });
    }
}

}  // namespace sbli
