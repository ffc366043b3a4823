// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "feh_internal.hpp"

namespace feh {

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Remap the hardware block id so that every XCD walks a
// contiguous range of logical tiles (neighbouring tiles share halos in L2).
__device__ __forceinline__ int xcd_remap(int id, int total) {
    constexpr int X = 8;
    const int xcd = id % X;
    const int k = id / X;
    const int q = total / X, r = total % X;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// Periodic index; the common case (one period away at most) avoids a division.
__device__ __forceinline__ int wrap(int i, int n) {
    if (i >= n) {
        i -= n;
        if (i >= n) i %= n;
    } else if (i < 0) {
        i += n;
        if (i < 0) {
            i %= n;
            if (i < 0) i += n;
        }
    }
    return i;
}

// Deterministic block sum of one double (fixed order), result in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        #pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += sh[i];
    }
    return s;
}

}  // namespace feh
