// Fixed-order workgroup sums for the norm stages.
#pragma once

#include <hip/hip_runtime.h>

namespace nmg {

// Binary-tree sum red[t] += red[t + h], h = COUNT / 2 .. 1, of COUNT (a power
// of two, at least 64) values in LDS, ready after a barrier.  The levels
// h >= 64 go through LDS with a barrier each; the last six run in wave 0 by
// cross-lane shifts, which add the same pairs in the same order, so the sum
// is the one of the all-LDS tree.  Every thread of the NT-thread workgroup
// calls it; thread 0 receives the sum.
template <int COUNT, int NT>
__device__ inline double tree_sum(double* red, int tid) {
    static_assert(COUNT >= 64 && (COUNT & (COUNT - 1)) == 0, "tree size");
#pragma unroll
    for (int h = COUNT / 2; h >= 64; h >>= 1) {
        for (int t = tid; t < h; t += NT) red[t] += red[t + h];
        __syncthreads();
    }
    double v = 0.0;
    if (tid < 64) {
        v = red[tid];
#pragma unroll
        for (int h = 32; h > 0; h >>= 1) v += __shfl_down(v, h, 64);
    }
    return v;
}

}  // namespace nmg
