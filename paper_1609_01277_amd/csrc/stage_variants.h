// Compiled launch variants of the fused stage kernel and their dispatch.
//
// A variant fixes the (x, y) tile of a workgroup and how far the global loads
// run ahead (see fused_stage_body).  Every variant performs the same arithmetic
// per point in the same order, so all of them give bitwise identical states;
// they differ only in speed, which the autotuner measures.
#pragma once

#include "kernels_stage_fused.h"

namespace sbli {

struct StageVariant {
    int tx, ty, pre, rot;
    int minw;   // wavefronts per SIMD the register allocation must allow (1 = as many VGPRs as needed)
    int db;     // 1: double-buffered LDS planes, one barrier per z-iteration
    int zl;     // 1: the R planes below the output plane in LDS instead of registers
};

// X-macro lists of (TX, TY, PRE, RT, MINW, DB, ZL) per (type, radius).  The first
// entry is the default before tuning.
#define SBLI_VARIANTS_D1(X) \
    X(16, 16, 1, 0, 1, 0, 0) X(16, 16, 1, 1, 1, 0, 0) X(32, 8, 1, 1, 1, 0, 0) X(16, 8, 1, 1, 2, 0, 0) X(16, 16, 1, 1, 1, 1, 0)
#define SBLI_VARIANTS_D2(X)                                                                                    \
    X(16, 16, 1, 0, 1, 0, 0) X(16, 16, 1, 1, 1, 0, 0) X(16, 16, 0, 1, 1, 0, 0) X(32, 8, 0, 0, 1, 0, 0) X(16, 8, 1, 1, 2, 0, 0) \
    X(16, 16, 1, 1, 1, 1, 0) X(16, 16, 1, 0, 1, 1, 0)
#define SBLI_VARIANTS_D3(X) X(8, 8, 0, 0, 1, 0, 0) X(8, 8, 1, 0, 1, 0, 0) X(16, 8, 1, 0, 1, 0, 0) X(16, 8, 1, 0, 1, 1, 0)
#define SBLI_VARIANTS_D4(X) \
    X(16, 4, 0, 0, 1, 0, 0) X(16, 4, 1, 0, 1, 0, 0) X(8, 8, 0, 0, 1, 0, 0) X(16, 4, 1, 0, 1, 0, 1) X(8, 8, 1, 0, 1, 0, 1)
#define SBLI_VARIANTS_F1(X) \
    X(16, 16, 1, 0, 1, 0, 0) X(16, 16, 1, 1, 1, 0, 0) X(32, 8, 1, 1, 1, 0, 0) X(16, 8, 1, 0, 1, 0, 0) X(16, 16, 1, 1, 1, 1, 0)
#define SBLI_VARIANTS_F2(X)                                                                                   \
    X(16, 8, 1, 0, 1, 0, 0) X(16, 8, 1, 1, 1, 0, 0) X(16, 16, 1, 1, 1, 0, 0) X(32, 8, 1, 1, 1, 0, 0) X(32, 8, 1, 1, 3, 0, 0) \
    X(16, 16, 1, 1, 3, 0, 0) X(16, 16, 1, 1, 1, 1, 0) X(32, 8, 1, 1, 1, 1, 0) X(16, 16, 1, 1, 3, 1, 0)            \
    X(32, 16, 1, 1, 1, 0, 0) X(32, 16, 1, 1, 1, 1, 0)
#define SBLI_VARIANTS_F3(X) X(16, 16, 0, 0, 1, 0, 0) X(16, 16, 1, 0, 1, 0, 0) X(16, 8, 1, 0, 1, 0, 0)
#define SBLI_VARIANTS_F4(X) X(16, 8, 0, 0, 1, 0, 0) X(16, 8, 1, 0, 1, 0, 0) X(16, 4, 1, 0, 1, 0, 0)

// One launch: the boxes (device table), their total workgroup count, the mode
// and the RK coefficients.
struct StageArgs {
    hipStream_t stream;
    const void* inst;   // device array of BoxInst<T>
    int ninst;
    int total_wg;
    int mode;
    double dt_scale, A, B;
    int sym;            // 1 if a box of the launch has a symmetry axis
};

template <typename T, int R, int TX, int TY, int PRE, int RT, int MINW, int DB, int ZL, int MODE>
inline void launch_fused_cfg(const StageArgs& a, const T* qin, T* dq, T* qout) {
    if (a.sym)
        fused_stage_kernel<T, R, TX, TY, MODE, PRE, RT, MINW, 1, DB, ZL><<<dim3(a.total_wg), FusedShape<R, TX, TY>::NT,
                                                                       0, a.stream>>>(
            qin, dq, qout, (const BoxInst<T>*)a.inst, a.ninst, (T)a.dt_scale, (T)a.A, (T)a.B);
    else
        fused_stage_kernel<T, R, TX, TY, MODE, PRE, RT, MINW, 0, DB, ZL><<<dim3(a.total_wg), FusedShape<R, TX, TY>::NT,
                                                                       0, a.stream>>>(
            qin, dq, qout, (const BoxInst<T>*)a.inst, a.ninst, (T)a.dt_scale, (T)a.A, (T)a.B);
}

template <typename T, int R, int TX, int TY, int PRE, int RT, int MINW, int DB, int ZL>
inline bool try_variant(int& k, int want, const StageArgs& a, const T* qin, T* dq, T* qout) {
    if (k++ != want) return false;
    switch (a.mode) {
        case kModeRHS: launch_fused_cfg<T, R, TX, TY, PRE, RT, MINW, DB, ZL, kModeRHS>(a, qin, dq, qout); break;
        case kModeStage1: launch_fused_cfg<T, R, TX, TY, PRE, RT, MINW, DB, ZL, kModeStage1>(a, qin, dq, qout); break;
        case kModeStage2: launch_fused_cfg<T, R, TX, TY, PRE, RT, MINW, DB, ZL, kModeStage2>(a, qin, dq, qout); break;
        default: launch_fused_cfg<T, R, TX, TY, PRE, RT, MINW, DB, ZL, kModeStage3>(a, qin, dq, qout); break;
    }
    return true;
}

#define SBLI_TRY(TX_, TY_, PRE_, RT_, MINW_, DB_, ZL_) \
    if (try_variant<T, R, TX_, TY_, PRE_, RT_, MINW_, DB_, ZL_>(k, v, a, qin, dq, qout)) return true;
#define SBLI_ENTRY(TX_, TY_, PRE_, RT_, MINW_, DB_, ZL_) StageVariant{TX_, TY_, PRE_, RT_, MINW_, DB_, ZL_},

template <typename T, int R>
struct VariantSet;

// The launch function of a (type, radius) -- which instantiates its kernels --
// is defined only in the translation unit stage_{f64,f32}_r{1..4}.hip that sets
// SBLI_STAGE_TU_{TYPE,R,LIST}, so the variants compile in parallel.
#define SBLI_VARIANT_SET(TYPE, RR, LIST)                                                                  \
    template <>                                                                                           \
    struct VariantSet<TYPE, RR> {                                                                         \
        using T = TYPE;                                                                                   \
        static constexpr int R = RR;                                                                      \
        static int count() {                                                                              \
            static const StageVariant t[] = {LIST(SBLI_ENTRY)};                                          \
            return (int)(sizeof(t) / sizeof(t[0]));                                                       \
        }                                                                                                 \
        static StageVariant get(int i) {                                                                  \
            static const StageVariant t[] = {LIST(SBLI_ENTRY)};                                          \
            return t[i];                                                                                  \
        }                                                                                                 \
        static bool launch(int v, const StageArgs& a, const T* qin, T* dq, T* qout);                  \
    };

SBLI_VARIANT_SET(double, 1, SBLI_VARIANTS_D1)
SBLI_VARIANT_SET(double, 2, SBLI_VARIANTS_D2)
SBLI_VARIANT_SET(double, 3, SBLI_VARIANTS_D3)
SBLI_VARIANT_SET(double, 4, SBLI_VARIANTS_D4)
SBLI_VARIANT_SET(float, 1, SBLI_VARIANTS_F1)
SBLI_VARIANT_SET(float, 2, SBLI_VARIANTS_F2)
SBLI_VARIANT_SET(float, 3, SBLI_VARIANTS_F3)
SBLI_VARIANT_SET(float, 4, SBLI_VARIANTS_F4)

#if defined(SBLI_STAGE_TU_TYPE) && defined(SBLI_STAGE_TU_R) && defined(SBLI_STAGE_TU_LIST)
bool VariantSet<SBLI_STAGE_TU_TYPE, SBLI_STAGE_TU_R>::launch(int v, const StageArgs& a, const T* qin, T* dq,
                                                             T* qout) {
    int k = 0;
    SBLI_STAGE_TU_LIST(SBLI_TRY)
    return false;
}
#endif

#undef SBLI_TRY
#undef SBLI_ENTRY
#undef SBLI_VARIANT_SET

// Runtime dispatch over (radius, variant) for one element type.
template <typename T>
struct StageDispatch {
    static int count(int r);
    static StageVariant get(int r, int i);
    static bool launch(int r, int v, const StageArgs& a, const T* qin, T* dq, T* qout);
};

template <typename T>
inline int StageDispatch<T>::count(int r) {
    switch (r) {
        case 1: return VariantSet<T, 1>::count();
        case 2: return VariantSet<T, 2>::count();
        case 3: return VariantSet<T, 3>::count();
        default: return VariantSet<T, 4>::count();
    }
}
template <typename T>
inline StageVariant StageDispatch<T>::get(int r, int i) {
    switch (r) {
        case 1: return VariantSet<T, 1>::get(i);
        case 2: return VariantSet<T, 2>::get(i);
        case 3: return VariantSet<T, 3>::get(i);
        default: return VariantSet<T, 4>::get(i);
    }
}
template <typename T>
inline bool StageDispatch<T>::launch(int r, int v, const StageArgs& a, const T* qin, T* dq, T* qout) {
    switch (r) {
        case 1: return VariantSet<T, 1>::launch(v, a, qin, dq, qout);
        case 2: return VariantSet<T, 2>::launch(v, a, qin, dq, qout);
        case 3: return VariantSet<T, 3>::launch(v, a, qin, dq, qout);
        default: return VariantSet<T, 4>::launch(v, a, qin, dq, qout);
    }
}

// Fills the launch-geometry part of a box entry for tile (tx, ty) and zchunk;
// returns the number of workgroups the box takes.
template <typename T>
inline int set_box_geometry(BoxInst<T>& b, int tx, int ty, int zchunk, int first_wg) {
    b.tiles_x = (b.c.n[0] + tx - 1) / tx;
    b.tiles_y = (b.c.n[1] + ty - 1) / ty;
    b.zchunk = zchunk;
    b.first_wg = first_wg;
    b.num_wg = b.tiles_x * b.tiles_y * ((b.c.n[2] + zchunk - 1) / zchunk);
    return b.num_wg;
}

}  // namespace sbli
