// Shared device-side definitions of libsbli: per-solve constants and helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sbli {

constexpr int kMaxR = 4;   // largest supported stencil radius (order 8)

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
};

enum StageMode { kModeRHS = 0, kModeStage1 = 1, kModeStage2 = 2, kModeStage3 = 3 };

// Index of the neighbour `m` points away along `axis` (periodic), given the
// point's coordinate `c` on that axis, its linear index `id` and the axis
// stride.  Requires |m| < n.
__device__ __forceinline__ int64_t shifted(int64_t id, int c, int m, int n, int64_t stride) {
    int cc = c + m;
    cc = cc >= n ? cc - n : (cc < 0 ? cc + n : cc);
    return id + (int64_t)(cc - c) * stride;
}

}  // namespace sbli
