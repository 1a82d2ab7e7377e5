// Launches of the staged form of the stage kernel (kernels_staged.h) for every
// element type, radius 1..6 and mode; compiled in a translation unit of its own.
#include "kernels_staged.h"
#include "staged.h"

namespace sbli {

template <typename T, int R>
static void staged_run(const StagedArgs& a, const T* qin, T* dq, T* qout, T* nf) {
    const BoxConst<T>& c = *(const BoxConst<T>*)a.box;
    auto grid_of = [&](int tiles, int zc) {
        const int64_t units = (int64_t)tiles * ((c.n[2] + zc - 1) / zc);
        return (unsigned)(kStagedXcds * ((units + kStagedXcds - 1) / kStagedXcds));
    };
    {
        // The nested-field step in 32x32 tiles where the register and LDS budget allows
        // (every radius in FP32, up to R = 4 in FP64): each tile then fetches its R-wide
        // x-arms, 32-byte row pieces of 128-byte lines, for four times as many own points.
        constexpr int TN = (sizeof(T) == 8 && R > 4) ? kStagedTile : 2 * kStagedTile;
        const int tx = (c.n[0] + TN - 1) / TN, ty = (c.n[1] + TN - 1) / TN;
        const int zn = kNestedRun;
        staged_nested_zring_kernel<T, R, TN><<<grid_of(tx * ty, zn), TN * TN, 0, a.stream>>>(qin, nf, c, tx, ty, zn);
    }
    const int tx = (c.n[0] + kStagedTile - 1) / kStagedTile, ty = (c.n[1] + kStagedTile - 1) / kStagedTile;
    constexpr int NT = kStagedTile * kStagedTile;
    const T dt = (T)a.dt, A = (T)a.A, B = (T)a.B;
    const T* clos = (const T*)a.clos;
    const int zc = 1;   // one plane per workgroup: see staged_unit
    const unsigned grid = grid_of(tx * ty, zc);
    switch (a.mode) {
        case kModeRHS:
            staged_tiled_kernel<T, R, kModeRHS><<<grid, NT, 0, a.stream>>>(qin, nf, dq, qout, c, dt, A, B, clos,
                                                                           a.cflag, tx, ty, zc);
            break;
        case kModeStage1:
            staged_tiled_kernel<T, R, kModeStage1><<<grid, NT, 0, a.stream>>>(qin, nf, dq, qout, c, dt, A, B, clos,
                                                                              a.cflag, tx, ty, zc);
            break;
        case kModeStage2:
            staged_tiled_kernel<T, R, kModeStage2><<<grid, NT, 0, a.stream>>>(qin, nf, dq, qout, c, dt, A, B, clos,
                                                                              a.cflag, tx, ty, zc);
            break;
        default:
            staged_tiled_kernel<T, R, kModeStage3><<<grid, NT, 0, a.stream>>>(qin, nf, dq, qout, c, dt, A, B, clos,
                                                                              a.cflag, tx, ty, zc);
            break;
    }
}

template <typename T>
static void staged_dispatch(const StagedArgs& a, const void* qin, void* dq, void* qout) {
    T* nf = (T*)a.scratch;
    const T* qi = (const T*)qin;
    T* d = (T*)dq;
    T* qo = (T*)qout;
    switch (a.r) {
        case 1: staged_run<T, 1>(a, qi, d, qo, nf); break;
        case 2: staged_run<T, 2>(a, qi, d, qo, nf); break;
        case 3: staged_run<T, 3>(a, qi, d, qo, nf); break;
        case 4: staged_run<T, 4>(a, qi, d, qo, nf); break;
        case 5: staged_run<T, 5>(a, qi, d, qo, nf); break;
        default: staged_run<T, 6>(a, qi, d, qo, nf); break;
    }
}

void staged_launch(const StagedArgs& a, const void* qin, void* dq, void* qout) {
    if (a.f64) staged_dispatch<double>(a, qin, dq, qout);
    else staged_dispatch<float>(a, qin, dq, qout);
}

}  // namespace sbli
