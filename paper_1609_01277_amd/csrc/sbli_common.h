// Shared device-side definitions of libsbli: per-solve constants and helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sbli {

constexpr int kMaxR = 6;   // largest supported stencil radius (order 12)

// Constants of one periodic box, pre-scaled so the kernels never divide by the
// grid spacing (paper Sec. "Code generation": rationals and reciprocals such as
// 1/Re are evaluated once and stored).
template <typename T>
struct BoxConst {
    int n[3];                 // points per axis (x, y, z)
    int64_t P;                // n0 * n1 * n2
    T da[3][kMaxR];           // a_m / h_axis         (first derivative)
    T d2c0[3];                // c_0 / h_axis^2       (second derivative)
    T d2c[3][kMaxR];          // c_m / h_axis^2
    T gm1;                    // gamma - 1
    T gM2;                    // gamma * M^2          (T = gamma M^2 p / rho)
    T inv_Re;                 // 1 / Re
    T inv_3Re;                // 1 / (3 Re)
    T kappa;                  // 1 / ((gamma - 1) M^2 Pr Re), mu = 1
    T inv_Re23;               // 2 / (3 Re)
    int sym[3];               // per axis: 1 = symmetry boundaries, 0 = periodic
};

// Index of point v (-n <= v < 2n) on an axis of n points: wrapped on a periodic
// axis; mirrored on a symmetry axis (n -> n-1, n+1 -> n-2, -1 -> 0, -2 -> 1),
// where `flip` becomes the sign-bit mask 0x80000000 for a mirrored point (a
// vector component normal to the boundary changes sign there), else 0.
__device__ __forceinline__ int map_index(int v, int n, int sym, unsigned& flip) {
    flip = 0u;
    if (sym) {
        if (v < 0) { v = -1 - v; flip = 0x80000000u; }
        else if (v >= n) { v = 2 * n - 1 - v; flip = 0x80000000u; }
        return v;
    }
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// The same for any v: a symmetry axis continues with period 2n (the doubled,
// mirrored box), so v is first reduced modulo 2n (modulo n when periodic).
__device__ __forceinline__ int fold_index(int v, int n, int sym, unsigned& flip) {
    flip = 0u;
    const int period = sym ? 2 * n : n;
    int t = v % period;
    if (t < 0) t += period;
    if (sym && t >= n) {
        t = 2 * n - 1 - t;
        flip = 0x80000000u;
    }
    return t;
}

// v with its sign bit toggled by `mask` (0 or 0x80000000): exact negation.
__device__ __forceinline__ double flip_sign(double v, unsigned mask) {
    return __hiloint2double(__double2hiint(v) ^ (int)mask, __double2loint(v));
}
__device__ __forceinline__ float flip_sign(float v, unsigned mask) {
    return __int_as_float(__float_as_int(v) ^ (int)mask);
}

enum StageMode { kModeRHS = 0, kModeStage1 = 1, kModeStage2 = 2, kModeStage3 = 3 };

// Index of the neighbour `m` points away along an axis (periodic, or mirrored
// when sym), given the point's coordinate `c` on that axis, its linear index
// `id` and the axis stride.  Requires |m| <= n.
__device__ __forceinline__ int64_t shifted(int64_t id, int c, int m, int n, int64_t stride, int sym = 0) {
    unsigned flip;
    const int cc = map_index(c + m, n, sym, flip);
    return id + (int64_t)(cc - c) * stride;
}

}  // namespace sbli
