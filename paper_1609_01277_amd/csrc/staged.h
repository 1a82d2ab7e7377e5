// Host interface of the staged form of the stage kernel (staged.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace sbli {

// Scratch words per point the staged form needs: the 6 nested fields.
constexpr int kStagedScratchWords = 6;

struct StagedArgs {
    hipStream_t stream;
    bool f64;           // element type of the state: double (true) or float
    int r;              // stencil radius, 1..6
    const void* box;    // host BoxConst<T> of the box (passed to the kernels by value)
    void* scratch;      // device, kStagedScratchWords * P elements
    int mode;           // StageMode
    double dt, A, B;
    const void* clos;   // device closure term (5 planar fields, the state's type) or null
    const int* cflag;   // device flag: the closure is added only while *cflag != 0
};

// Enqueues the two launches of one residual / RK3 stage on a.stream.
void staged_launch(const StagedArgs& a, const void* qin, void* dq, void* qout);

}  // namespace sbli
