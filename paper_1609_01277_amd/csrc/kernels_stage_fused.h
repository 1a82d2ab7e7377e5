// Fused residual + RK3-stage kernel: one launch per stage, the state read once
// and written once per point (plus dq).
//
// Data flow (per workgroup): a TX x TY tile of (x, y) columns marches along z.
// The nested terms of the residual (viscous work D_j(u_i tau_ij) and the
// grad-div part D_i(D_k u_k), paper Sec. "Expanding": inner derivative first)
// need the velocity gradient on a ring of R columns around the tile and R
// planes ahead of the output plane, so every stage is a three-step pipeline per
// z-plane:
//   1. each column thread loads the state R planes ahead of the gradient plane
//      and keeps a register window of 3R+1 planes of point fields
//      (rho, rho u_i, rho E, u_i, p, T);
//   2. the "gradient" plane a: velocity gradient by x/y stencils over an LDS
//      plane of u (tile + 2R ring) and z stencils over the register window,
//      reduced at once to the six fields the outer derivatives act on
//      (V_j = u_i tau_ij and theta - D_j u_j), kept in register windows;
//   3. the output plane o = a - R: every x/y derivative from an LDS plane of
//      point fields (tile + R ring), every z derivative from the register
//      windows, the residual, and the RK update written straight to HBM.
// Columns of the R-ring around the tile are handled by extra "halo" threads
// (whole wavefronts apart from the interior ones); the 2R-ring of u needed only
// for the x/y gradient stencils of halo columns is loaded directly.
//
// Two barrier schedules.  DB = 0: step 1 | barrier | step 2 | barrier | step 3,
// each LDS plane single-buffered.  DB = 1: the LDS planes of u and of the point
// fields alternate between two buffers by iteration parity and the point fields
// of the output plane are stored in step 1.  Step 3 then reads nothing that
// another thread writes in the same iteration (the z-nested fields of the newest
// gradient plane belong to the thread's own column), so one barrier per
// iteration suffices: the residual of plane o overlaps the gradients and, in the
// halo wavefronts, the loads of the next iteration.  Periodic
// wrap (or, on a symmetry axis, the mirror image with the normal momentum
// negated) is folded into the column and plane coordinates, so ragged tiles and
// boundaries need no special case beyond masking the stores.
#pragma once

#include <type_traits>
#include <utility>

#include "sbli_common.h"

namespace sbli {

template <int R, int TX, int TY>
struct FusedShape {
    static constexpr int NI = TX * TY;              // interior columns
    static constexpr int NHX = 2 * R * TY;          // x-ring columns
    static constexpr int NHY = 2 * R * TX;          // y-ring columns
    static constexpr int NE1 = NI + NHX + NHY;      // columns with a register window
    static constexpr int NT = (NE1 + 63) / 64 * 64; // threads per workgroup
    static constexpr int BX1 = TX + 2 * R, BY1 = TY + 2 * R;  // LDS box of point fields
    static constexpr int BX2 = TX + 4 * R, BY2 = TY + 4 * R;  // LDS box of u
    static constexpr int NOUT = 2 * R * TY + 2 * R * TX + 4 * R * R;  // u-only ring points
    static_assert(NI % 64 == 0, "interior columns must fill whole wavefronts");
    static_assert(NOUT <= NT, "one u-ring point per thread at most");
};

// Point fields kept per plane and per column.
template <typename T>
struct PF {
    T rho, m0, m1, m2, E, u0, u1, u2, p, Tm;
};

// 1/x from the hardware reciprocal refined by Newton steps (two in FP64, one in
// FP32): within an ulp of the quotient, at a third of the instructions of the
// IEEE division sequence.
__device__ __forceinline__ double fast_recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fast_recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// a*b + c with one rounding.  The residual arithmetic spells out its fused
// multiply-adds (the library is built with contraction limited to single
// expressions), so every launch variant rounds every point identically.
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ PF<T> make_pf(T rho, T m0, T m1, T m2, T E, T gm1, T gM2) {
    PF<T> s;
    s.rho = rho;
    s.m0 = m0;
    s.m1 = m1;
    s.m2 = m2;
    s.E = E;
    const T rr = fast_recip(rho);
    s.u0 = m0 * rr;
    s.u1 = m1 * rr;
    s.u2 = m2 * rr;
    const T ke2 = fmaT(m2, s.u2, fmaT(m1, s.u1, m0 * s.u0));    // 2 x kinetic energy
    s.p = gm1 * fmaT(T(-0.5), ke2, E);
    s.Tm = gM2 * s.p * rr;
    return s;
}

// Calls f(integral_constant<int, 0>), ..., f(integral_constant<int, N-1>).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// n stores that the hardware drops (a buffer descriptor of one element and an
// offset beyond it): they keep the count of memory operations equal on both
// sides of a branch (see step 4 of fused_stage_body).
constexpr int kDropOff = (int)0x80000000;
constexpr int kBufferWord3 = 0x00020000;   // descriptor word 3 of a raw (untyped) buffer
typedef int sbli_v2i __attribute__((ext_vector_type(2)));
template <int N, typename T>
__device__ __forceinline__ void dropped_stores(T* any) {
    const __amdgpu_buffer_rsrc_t d = __builtin_amdgcn_make_buffer_rsrc(any, 0, (int)sizeof(T), kBufferWord3);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(sbli_v2i{0, 0}, d, kDropOff, 0, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(0, d, kDropOff, 0, 0);
    }
}

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Number of LDS fields of the output plane (the point fields).
constexpr int kPlFields = 10;

// Accumulates, for one direction d, the derivative sums of the residual from a
// neighbour pair (a = +m, b = -m) with weights w (first) and w2 (second).
template <typename T>
struct DirSums {
    T dRho, dM0, dM1, dM2, dF0, dF1, dF2, dE, dH, dU, dTh, d2U0, d2U1, d2U2, d2T;
    __device__ __forceinline__ void zero() {
        dRho = dM0 = dM1 = dM2 = dF0 = dF1 = dF2 = dE = dH = dU = dTh = 0;
        d2U0 = d2U1 = d2U2 = d2T = 0;
    }
    // d is the direction (0, 1, 2): selects u_d and which momentum gets 2p.
    template <int d>
    __device__ __forceinline__ void add(const PF<T>& a, T Va, T Tha, const PF<T>& b, T Vb, T Thb, T w, T w2) {
        const T ua = d == 0 ? a.u0 : (d == 1 ? a.u1 : a.u2);
        const T ub = d == 0 ? b.u0 : (d == 1 ? b.u1 : b.u2);
        dRho = fmaT(w, a.rho - b.rho, dRho);
        dM0 = fmaT(w, a.m0 - b.m0, dM0);
        dM1 = fmaT(w, a.m1 - b.m1, dM1);
        dM2 = fmaT(w, a.m2 - b.m2, dM2);
        // momentum fluxes rho u_i u_d (+ 2p for i = d): differences a - b
        const T pa2 = T(2) * (a.p - b.p);
        const T f0 = d == 0 ? fmaT(a.m0, ua, pa2 - b.m0 * ub) : fmaT(a.m0, ua, -(b.m0 * ub));
        const T f1 = d == 1 ? fmaT(a.m1, ua, pa2 - b.m1 * ub) : fmaT(a.m1, ua, -(b.m1 * ub));
        const T f2 = d == 2 ? fmaT(a.m2, ua, pa2 - b.m2 * ub) : fmaT(a.m2, ua, -(b.m2 * ub));
        dF0 = fmaT(w, f0, dF0);
        dF1 = fmaT(w, f1, dF1);
        dF2 = fmaT(w, f2, dF2);
        dE = fmaT(w, a.E - b.E, dE);
        // energy flux (rho E + 2p) u_d - 2 V_d: difference a - b
        const T hb = fmaT(fmaT(T(2), b.p, b.E), ub, T(-2) * Vb);
        const T fh = fmaT(fmaT(T(2), a.p, a.E), ua, fmaT(T(-2), Va, -hb));
        dH = fmaT(w, fh, dH);
        dU = fmaT(w, ua - ub, dU);
        dTh = fmaT(w, Tha - Thb, dTh);
        d2U0 = fmaT(w2, a.u0 + b.u0, d2U0);
        d2U1 = fmaT(w2, a.u1 + b.u1, d2U1);
        d2U2 = fmaT(w2, a.u2 + b.u2, d2U2);
        d2T = fmaT(w2, a.Tm + b.Tm, d2T);
    }
    // Adds this direction's part of the residual (paper eq. mass, momentum,
    // energy in the skew-symmetric form, regrouped by linearity) at point s.
    template <int d>
    __device__ __forceinline__ void finish(const PF<T>& s, T c0, const BoxConst<T>& c, T& Rr, T& R0, T& R1, T& R2,
                                           T& RE) {
        const T ud = d == 0 ? s.u0 : (d == 1 ? s.u1 : s.u2);
        const T e0 = fmaT(c0, s.u0, d2U0);
        const T e1 = fmaT(c0, s.u1, d2U1);
        const T e2 = fmaT(c0, s.u2, d2U2);
        const T eT = fmaT(c0, s.Tm, d2T);
        const T dMd = d == 0 ? dM0 : (d == 1 ? dM1 : dM2);
        const T h = T(-0.5);
        Rr = fmaT(h, dMd + fmaT(ud, dRho, s.rho * dU), Rr);
        R0 = fmaT(c.inv_Re, e0, fmaT(h, dF0 + fmaT(ud, dM0, s.m0 * dU), R0));
        R1 = fmaT(c.inv_Re, e1, fmaT(h, dF1 + fmaT(ud, dM1, s.m1 * dU), R1));
        R2 = fmaT(c.inv_Re, e2, fmaT(h, dF2 + fmaT(ud, dM2, s.m2 * dU), R2));
        const T ed = d == 0 ? e0 : (d == 1 ? e1 : e2);
        if (d == 0) R0 = fmaT(c.inv_3Re, ed + dTh, R0);
        if (d == 1) R1 = fmaT(c.inv_3Re, ed + dTh, R1);
        if (d == 2) R2 = fmaT(c.inv_3Re, ed + dTh, R2);
        RE = fmaT(c.kappa, eT, fmaT(h, dH + fmaT(ud, dE, s.E * dU), RE));
    }
};

// One workgroup = one (x, y) tile and one z-chunk [z0, z0 + zc).
// PRE: whether the state of the entering plane and of the u-ring point is
// requested one iteration ahead (1) or in the iteration itself (0).  RT = 1
// rotates the register window instead of shifting it (for windows of at most 7
// planes).
// clos (may be null): a closure term with the state's planar layout, added to
// the residual when *cflag != 0.
template <typename T, int R, int TX, int TY, int MODE, int PRE, int RT, int SYM, int DB, int ZL>
__device__ __forceinline__ void fused_stage_body(const T* __restrict__ q, T* __restrict__ dq, T* __restrict__ out,
                                                 const BoxConst<T>& c, int x0, int y0, int z0, int zc, T dt, T A,
                                                 T B, const T* __restrict__ clos, const int* __restrict__ cflag) {
    using S = FusedShape<R, TX, TY>;
    constexpr int NB = DB ? 2 : 1;     // buffers of the u plane and the point-field plane
    __shared__ T s_u[NB][3][S::BY2][S::BX2];
    __shared__ T s_pl[NB][kPlFields][S::BY1][S::BX1];
    // Rings of the nested-derivative fields, indexed by iteration: (V_x, Th_x,
    // V_y, Th_y) of the last R+1 gradient planes over the tile and its R-ring,
    // and (V_z, Th_z) of the last 2R+1 gradient planes over the tile.
    __shared__ T s_axy[R + 1][4][S::BY1][S::BX1];
    __shared__ T s_az[2 * R + 1][2][TY][TX];
    // ZL: the point fields of the R planes below the output plane (own column,
    // stored when a plane leaves the centre of the window) are kept in LDS
    // instead of the register window, which then needs 2R + 1 live planes.
    __shared__ T s_zt[ZL ? R : 1][ZL ? kPlFields : 1][ZL ? TY : 1][ZL ? TX : 1];

    const int nx = c.n[0], ny = c.n[1], nz = c.n[2];
    const int64_t P = c.P;
    const int64_t plane = (int64_t)nx * ny;
    const int tid = threadIdx.x;

    // ---- column role and coordinates ----
    int cx = 0, cy = 0;
    const bool e1 = tid < S::NE1;
    const bool interior = tid < S::NI;
    if (tid < S::NI) {
        cx = tid % TX;
        cy = tid / TX;
    } else if (tid < S::NI + S::NHX) {
        const int t = tid - S::NI;
        const int side = t / (R * TY);
        const int t2 = t % (R * TY);
        cy = t2 / R;
        const int k = t2 % R;
        cx = side ? TX + k : -R + k;
    } else if (tid < S::NE1) {
        const int t = tid - S::NI - S::NHX;
        const int side = t / (R * TX);
        const int t2 = t % (R * TX);
        const int k = t2 / TX;
        cx = t2 % TX;
        cy = side ? TY + k : -R + k;
    }
    // Periodic axes wrap; symmetry axes mirror, and a mirrored column carries the
    // sign-bit mask of the momentum component normal to that boundary.
    // SYM = 0 compiles the periodic case only (no masks, no sign flips).
    const int symx = SYM ? c.sym[0] : 0, symy = SYM ? c.sym[1] : 0, symz = SYM ? c.sym[2] : 0;
    unsigned fcx, fcy;
    const int64_t col = (int64_t)fold_index(y0 + cy, ny, symy, fcy) * nx + fold_index(x0 + cx, nx, symx, fcx);
    const bool store = interior && (x0 + cx < nx) && (y0 + cy < ny);

    // u-only ring point of this thread (if any): E2 minus E1.
    int ox = 0, oy = 0;
    const bool has_out = tid < S::NOUT;
    if (has_out) {
        int t = tid;
        if (t < 2 * R * TY) {                       // left / right, interior rows
            const int side = t / (R * TY);
            const int t2 = t % (R * TY);
            oy = t2 / R;
            const int k = t2 % R;
            ox = side ? TX + R + k : -2 * R + k;
        } else if ((t -= 2 * R * TY) < 2 * R * TX) {  // bottom / top, interior columns
            const int side = t / (R * TX);
            const int t2 = t % (R * TX);
            const int k = t2 / TX;
            ox = t2 % TX;
            oy = side ? TY + R + k : -2 * R + k;
        } else {                                    // the four R x R corners
            t -= 2 * R * TX;
            const int corner = t / (R * R);
            const int t2 = t % (R * R);
            const int ky = t2 / R, kx = t2 % R;
            ox = (corner & 1) ? TX + kx : -R + kx;
            oy = (corner & 2) ? TY + ky : -R + ky;
        }
    }
    unsigned fox, foy;
    const int64_t ocol = (int64_t)fold_index(y0 + oy, ny, symy, foy) * nx + fold_index(x0 + ox, nx, symx, fox);

    // ---- register windows ----
    constexpr int W = 3 * R + 1;
    constexpr bool ROT = RT && W <= 7;  // rotate instead of shifting (code size grows W-fold)
    PF<T> Qb[W];                  // point fields, planes L-3R .. L (logical index 3R = newest)
#pragma unroll
    for (int s = 0; s <= 3 * R; ++s) Qb[s] = PF<T>{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

    const int iters = zc + 4 * R;
    // With PRE = 1 the loads of iteration it+1 are issued before the work of
    // iteration it starts, and consumed one iteration later.
    T pq0 = 0, pq1 = 0, pq2 = 0, pq3 = 0, pq4 = 0;   // next q (own column)
    T pr0 = 1, pr1 = 0, pr2 = 0, pr3 = 0;            // next ring point (rho, rho u_i)
    // Sign-bit masks of the z-momentum of the planes just requested (mirror
    // images beyond a z symmetry boundary).  The loaded values stay untouched
    // until they are used, so a prefetch never waits for its data.
    unsigned pqz = 0u, prz = 0u;
    // planes stay within [-2R, nz + 2R): one mirror or wrap at most.  Every lane
    // loads in every iteration, from an in-range point (a lane without a column
    // reads the tile's first column; its values are unused).
    auto issue = [&](int it) {
        const int L = z0 - 2 * R + it;
        {
            const T* b = q + (int64_t)map_index(L, nz, symz, pqz) * plane + col;
            pq0 = b[0];
            pq1 = b[P];
            pq2 = b[2 * P];
            pq3 = b[3 * P];
            pq4 = b[4 * P];
        }
        {
            // the ring plane L - R is needed from the first gradient plane on
            const T* b = q + (int64_t)map_index(it >= 2 * R ? L - R : L, nz, symz, prz) * plane + ocol;
            pr0 = b[0];
            pr1 = b[P];
            pr2 = b[2 * P];
            pr3 = b[3 * P];
        }
    };
    if (PRE > 0) issue(0);
    // One z-iteration.  With ROT the window is never shifted: logical plane k of
    // the window lives in register slot (k + PH) % W, and the loop is unrolled W
    // times so every slot index is a compile-time constant.
    auto body = [&](auto ph, const int it) {
        constexpr int PH = decltype(ph)::value;
        auto slot = [](int k) { return ROT ? (k + PH) % W : k; };
            const int L = z0 - 2 * R + it;           // plane loaded this iteration
            const int bsel = DB ? (it & 1) : 0;      // LDS buffer of this iteration's planes
            if (PRE == 0) issue(it);
            const T cq0 = pq0, cq1 = flip_sign(pq1, fcx), cq2 = flip_sign(pq2, fcy), cq3 = flip_sign(pq3, pqz),
                    cq4 = pq4;
            const T cr0 = pr0, cr1 = flip_sign(pr1, fox), cr2 = flip_sign(pr2, foy), cr3 = flip_sign(pr3, prz);
            if (PRE > 0 && it + 1 < iters) issue(it + 1);
            __builtin_amdgcn_sched_barrier(0);
            // 1. plane L enters the window
            if (e1) {
                const PF<T> f = make_pf<T>(cq0, cq1, cq2, cq3, cq4, c.gm1, c.gM2);
                if (!ROT) {
    #pragma unroll
                    for (int s = 0; s < 3 * R; ++s) Qb[slot(s)] = Qb[slot(s + 1)];
                }
                Qb[slot(3 * R)] = f;
            }
            const bool do_grad = it >= 2 * R;
            const bool do_out = it >= 4 * R;
            // 2. LDS plane of u at the gradient plane a = L - R
            if (do_grad) {
                if (e1) {
                    s_u[bsel][0][cy + 2 * R][cx + 2 * R] = Qb[slot(2 * R)].u0;
                    s_u[bsel][1][cy + 2 * R][cx + 2 * R] = Qb[slot(2 * R)].u1;
                    s_u[bsel][2][cy + 2 * R][cx + 2 * R] = Qb[slot(2 * R)].u2;
                }
                if (has_out) {
                    const T rr = fast_recip(cr0);
                    s_u[bsel][0][oy + 2 * R][ox + 2 * R] = cr1 * rr;
                    s_u[bsel][1][oy + 2 * R][ox + 2 * R] = cr2 * rr;
                    s_u[bsel][2][oy + 2 * R][ox + 2 * R] = cr3 * rr;
                }
            }
            // LDS plane of point fields at the output plane o = L - 2R
            auto store_pl = [&]() {
                const PF<T>& f = Qb[slot(R)];
                const int ly = cy + R, lx = cx + R;
                s_pl[bsel][0][ly][lx] = f.rho;
                s_pl[bsel][1][ly][lx] = f.m0;
                s_pl[bsel][2][ly][lx] = f.m1;
                s_pl[bsel][3][ly][lx] = f.m2;
                s_pl[bsel][4][ly][lx] = f.E;
                s_pl[bsel][5][ly][lx] = f.u0;
                s_pl[bsel][6][ly][lx] = f.u1;
                s_pl[bsel][7][ly][lx] = f.u2;
                s_pl[bsel][8][ly][lx] = f.p;
                s_pl[bsel][9][ly][lx] = f.Tm;
            };
            if (DB && do_out && e1) store_pl();
            __syncthreads();
            // 3. velocity gradient at plane a -> nested fields
            if (do_grad && e1) {
                T g[3][3];
    #pragma unroll
                for (int b = 0; b < 3; ++b) {
                    T sx = 0, sy = 0, sz = 0;
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        sx = fmaT(c.da[0][m - 1],
                                  s_u[bsel][b][cy + 2 * R][cx + 2 * R + m] - s_u[bsel][b][cy + 2 * R][cx + 2 * R - m], sx);
                        sy = fmaT(c.da[1][m - 1],
                                  s_u[bsel][b][cy + 2 * R + m][cx + 2 * R] - s_u[bsel][b][cy + 2 * R - m][cx + 2 * R], sy);
                        const T up = b == 0 ? Qb[slot(2 * R + m)].u0 : (b == 1 ? Qb[slot(2 * R + m)].u1 : Qb[slot(2 * R + m)].u2);
                        const T um = b == 0 ? Qb[slot(2 * R - m)].u0 : (b == 1 ? Qb[slot(2 * R - m)].u1 : Qb[slot(2 * R - m)].u2);
                        sz = fmaT(c.da[2][m - 1], up - um, sz);
                    }
                    g[b][0] = sx;
                    g[b][1] = sy;
                    g[b][2] = sz;
                }
                const T uc[3] = {Qb[slot(2 * R)].u0, Qb[slot(2 * R)].u1, Qb[slot(2 * R)].u2};
                const T theta = g[0][0] + g[1][1] + g[2][2];
                T V[3];
    #pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    T v = 0;
    #pragma unroll
                    for (int ii = 0; ii < 3; ++ii) {
                        T tau = c.inv_Re * (g[ii][jj] + g[jj][ii]);
                        if (ii == jj) tau = fmaT(-c.inv_Re23, theta, tau);
                        v = fmaT(uc[ii], tau, v);
                    }
                    V[jj] = v;
                }
                const int sxy = it % (R + 1);
                s_axy[sxy][0][cy + R][cx + R] = V[0];
                s_axy[sxy][1][cy + R][cx + R] = theta - g[0][0];
                s_axy[sxy][2][cy + R][cx + R] = V[1];
                s_axy[sxy][3][cy + R][cx + R] = theta - g[1][1];
                if (interior) {
                    const int sz = it % (2 * R + 1);
                    s_az[sz][0][cy][cx] = V[2];   // read back only by this thread
                    s_az[sz][1][cy][cx] = theta - g[2][2];
                }
            }
            if (!DB) {
                if (do_out && e1) store_pl();
                __syncthreads();
            }
            // 4. residual and RK update at the output plane o = L - 2R.
            // The counter a wave waits on for its loads also counts its stores, and
            // the compiler (stores and loads may complete out of order) waits for it
            // to reach zero.  The next plane's prefetched state is therefore waited
            // for here, in every lane, before this plane's stores are issued: they
            // then drain during the next iteration instead of being waited for at
            // its start.  The global accesses of this step sit in branches (output
            // lanes, ragged tiles): a path that skips them is padded with as many
            // dropped stores, so that every lane's counter stays in step.
            if constexpr (PRE > 0) {
                asm volatile("" : "+v"(pq0), "+v"(pq1), "+v"(pq2), "+v"(pq3), "+v"(pq4));
                asm volatile("" : "+v"(pr0), "+v"(pr1), "+v"(pr2), "+v"(pr3));
            }
            constexpr int NLD = (MODE == kModeStage2 || MODE == kModeStage3) ? 5 : 0;
            constexpr int NST = (MODE == kModeRHS || MODE == kModeStage3) ? 5 : 10;
            if (do_out && interior) {
                const int ly = cy + R, lx = cx + R;
                const int64_t idx = (int64_t)(L - 2 * R) * plane + col;   // output planes lie inside the box
                T cd[5] = {0, 0, 0, 0, 0};
                if (NLD > 0) {
    #pragma unroll
                    for (int f = 0; f < 5; ++f) cd[f] = __builtin_nontemporal_load(&dq[f * P + idx]);
                }
                auto ld = [&](int yy, int xx) {
                    PF<T> f;
                    f.rho = s_pl[bsel][0][yy][xx];
                    f.m0 = s_pl[bsel][1][yy][xx];
                    f.m1 = s_pl[bsel][2][yy][xx];
                    f.m2 = s_pl[bsel][3][yy][xx];
                    f.E = s_pl[bsel][4][yy][xx];
                    f.u0 = s_pl[bsel][5][yy][xx];
                    f.u1 = s_pl[bsel][6][yy][xx];
                    f.u2 = s_pl[bsel][7][yy][xx];
                    f.p = s_pl[bsel][8][yy][xx];
                    f.Tm = s_pl[bsel][9][yy][xx];
                    return f;
                };
                const PF<T>& s = Qb[slot(R)];
                auto& axy = s_axy[(it - R) % (R + 1)];   // nested fields of plane o
                auto below = [&](int m) -> PF<T> {         // point fields of plane o - m
                    if constexpr (ZL) {
                        const int k = (it - m) % R;
                        PF<T> f;
                        f.rho = s_zt[k][0][cy][cx];
                        f.m0 = s_zt[k][1][cy][cx];
                        f.m1 = s_zt[k][2][cy][cx];
                        f.m2 = s_zt[k][3][cy][cx];
                        f.E = s_zt[k][4][cy][cx];
                        f.u0 = s_zt[k][5][cy][cx];
                        f.u1 = s_zt[k][6][cy][cx];
                        f.u2 = s_zt[k][7][cy][cx];
                        f.p = s_zt[k][8][cy][cx];
                        f.Tm = s_zt[k][9][cy][cx];
                        return f;
                    } else {
                        return Qb[slot(R - m)];
                    }
                };
                T Rr = 0, R0 = 0, R1 = 0, R2 = 0, RE = 0;
                {
                    DirSums<T> ds;
                    ds.zero();
    #pragma unroll
                    for (int m = 1; m <= R; ++m)
                        ds.template add<0>(ld(ly, lx + m), axy[0][ly][lx + m], axy[1][ly][lx + m], ld(ly, lx - m),
                                           axy[0][ly][lx - m], axy[1][ly][lx - m], c.da[0][m - 1], c.d2c[0][m - 1]);
                    ds.template finish<0>(s, c.d2c0[0], c, Rr, R0, R1, R2, RE);
                }
                {
                    DirSums<T> ds;
                    ds.zero();
    #pragma unroll
                    for (int m = 1; m <= R; ++m)
                        ds.template add<1>(ld(ly + m, lx), axy[2][ly + m][lx], axy[3][ly + m][lx], ld(ly - m, lx),
                                           axy[2][ly - m][lx], axy[3][ly - m][lx], c.da[1][m - 1], c.d2c[1][m - 1]);
                    ds.template finish<1>(s, c.d2c0[1], c, Rr, R0, R1, R2, RE);
                }
                {
                    DirSums<T> ds;
                    ds.zero();
    #pragma unroll
                    for (int m = 1; m <= R; ++m)
                        ds.template add<2>(Qb[slot(R + m)], s_az[(it + m - R) % (2 * R + 1)][0][cy][cx],
                                           s_az[(it + m - R) % (2 * R + 1)][1][cy][cx], below(m),
                                           s_az[(it - m - R) % (2 * R + 1)][0][cy][cx],
                                           s_az[(it - m - R) % (2 * R + 1)][1][cy][cx],
                                           c.da[2][m - 1], c.d2c[2][m - 1]);
                    ds.template finish<2>(s, c.d2c0[2], c, Rr, R0, R1, R2, RE);
                }
                if (store) {
                    // dq and the new state are streamed: nothing reads them again in
                    // this launch, so they need not displace the state in L2
                    T Rv[5] = {Rr, R0, R1, R2, RE};
                    if (clos != nullptr && cflag[0] != 0) {
    #pragma unroll
                        for (int f = 0; f < 5; ++f) Rv[f] += clos[f * P + idx];
                    }
                    const T qv[5] = {s.rho, s.m0, s.m1, s.m2, s.E};
    #pragma unroll
                    for (int f = 0; f < 5; ++f) {
                        if (MODE == kModeRHS) {
                            __builtin_nontemporal_store(Rv[f], &out[f * P + idx]);
                        } else {
                            T dn = dt * Rv[f];
                            if (MODE != kModeStage1) dn = fmaT(A, cd[f], dn);
                            if (MODE != kModeStage3) __builtin_nontemporal_store(dn, &dq[f * P + idx]);
                            __builtin_nontemporal_store(fmaT(B, dn, qv[f]), &out[f * P + idx]);
                        }
                    }
                } else {
                    dropped_stores<NST>(out);
                }
            } else {
                dropped_stores<NLD + NST>(out);
            }
            if constexpr (ZL) {
                // plane o leaves the centre of the window; only this thread reads it
                // back, as plane o' - m of the next R output planes
                if (interior && it >= 2 * R) {
                    const PF<T>& f = Qb[slot(R)];
                    const int k = it % R;
                    s_zt[k][0][cy][cx] = f.rho;
                    s_zt[k][1][cy][cx] = f.m0;
                    s_zt[k][2][cy][cx] = f.m1;
                    s_zt[k][3][cy][cx] = f.m2;
                    s_zt[k][4][cy][cx] = f.E;
                    s_zt[k][5][cy][cx] = f.u0;
                    s_zt[k][6][cy][cx] = f.u1;
                    s_zt[k][7][cy][cx] = f.u2;
                    s_zt[k][8][cy][cx] = f.p;
                    s_zt[k][9][cy][cx] = f.Tm;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
    };
    if constexpr (ROT) {
        for (int it0 = 0; it0 < iters; it0 += W) {
            static_for<W>([&](auto ph) {
                const int it = it0 + decltype(ph)::value;
                if (it < iters) body(ph, it);
            });
        }
    } else {
        for (int it = 0; it < iters; ++it) body(std::integral_constant<int, 0>{}, it);
    }
}

// One periodic box of a launch: its constants, where its state starts in the
// packed buffers, its time step and its share of the launch grid.
template <typename T>
struct BoxInst {
    BoxConst<T> c;
    int64_t offset;    // element offset of the box's state in q, dq and out
    T dt;              // time step (multiplied by the launch's dt_scale)
    int tiles_x, tiles_y, zchunk;
    int first_wg;      // first logical workgroup of this box
    int num_wg;        // tiles_x * tiles_y * ceil(nz / zchunk)
    const T* closure;  // closure term of this box (planar, 5 fields) or null
    const int* cflag;  // the closure is added only while *cflag != 0
};

// One launch covers `ninst` boxes (one for a single solver, many for an
// ensemble): a 1D grid whose logical workgroup ids are split between the boxes
// by first_wg.  Workgroups are handed to the 8 XCDs round-robin by id; the id is
// remapped so that each XCD (with its own L2) walks a contiguous run of
// neighbouring tiles, whose halos then hit in that L2.
// MINW: the fewest wavefronts per SIMD the register allocation must allow
// (2 caps a thread at 256 VGPRs, so two 4-wavefront workgroups share a CU).
// SYM: 1 for boxes with a symmetry axis, 0 for periodic boxes.
// DB: barrier schedule; ZL: lower planes of the window in LDS (see fused_stage_body).
template <typename T, int R, int TX, int TY, int MODE, int PRE, int RT, int MINW, int SYM, int DB, int ZL>
__global__ void __launch_bounds__((FusedShape<R, TX, TY>::NT), MINW)
    fused_stage_kernel(const T* __restrict__ q, T* __restrict__ dq, T* __restrict__ out,
                       const BoxInst<T>* __restrict__ inst, int ninst, T dt_scale, T A, T B) {
    const int total = gridDim.x;
    const int w = blockIdx.x;
    const int lam = (total % 8 == 0) ? (w % 8) * (total / 8) + w / 8 : w;
    int lo = 0, hi = ninst - 1;     // last box with first_wg <= lam
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (inst[mid].first_wg <= lam) lo = mid;
        else hi = mid - 1;
    }
    const BoxInst<T>& b = inst[lo];
    const int local = lam - b.first_wg;
    const int tile = local % (b.tiles_x * b.tiles_y);
    const int chunk = local / (b.tiles_x * b.tiles_y);
    const int tx = tile % b.tiles_x;
    const int ty = tile / b.tiles_x;
    const int z0 = chunk * b.zchunk;
    const int zc = min(b.zchunk, b.c.n[2] - z0);
    T* dqb = dq ? dq + b.offset : nullptr;
    fused_stage_body<T, R, TX, TY, MODE, PRE, RT, SYM, DB, ZL>(q + b.offset, dqb, out + b.offset, b.c, tx * TX, ty * TY, z0, zc,
                                              b.dt * dt_scale, A, B, b.closure, b.cflag);
}

}  // namespace sbli
