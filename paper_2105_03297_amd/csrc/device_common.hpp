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

// Element at a 32-bit byte offset from a base pointer: with the base uniform
// the load or store takes the scalar-base form (no 64-bit address arithmetic
// per access); the launchers check that the offsets fit.
template <typename P>
__device__ __forceinline__ P *at_byte(P *base, unsigned off) {
    return reinterpret_cast<P *>(reinterpret_cast<char *>(base) + off);
}
template <typename P>
__device__ __forceinline__ const P *at_byte(const P *base, unsigned off) {
    return reinterpret_cast<const P *>(reinterpret_cast<const char *>(base) + off);
}

// Raw buffer of `bytes` bytes from a uniform base (stride 0): a load or store
// takes a 32-bit per-lane byte offset and no 64-bit address arithmetic; an
// access at or past `bytes` is dropped (store) or reads zero (load), which
// lets a lane skip a store without a branch.  `bytes` < 2^31.
template <typename P>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(P *base, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(static_cast<const void *>(base)), (short)0, (int)bytes,
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T buffer_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte elements");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
}
template <typename T>
__device__ __forceinline__ void buffer_st(__amdgpu_buffer_rsrc_t r, unsigned off, T v) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
    } else {
        static_assert(sizeof(T) == 8, "4- or 8-byte elements");
        using U2 = __attribute__((ext_vector_type(2))) unsigned;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, 0);
    }
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
