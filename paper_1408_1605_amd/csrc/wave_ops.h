// Wave64 and workgroup primitives (device code).
#pragma once

#include "bfs_internal.h"

namespace bfsmi {

// Number of set bits of mask in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan over the 256 threads of a workgroup; *total receives the
// sum.  s_wave must hold kWG / 64 elements.  Contains two barriers: every
// thread of the workgroup must call it.
template <typename T>
__device__ __forceinline__ T wg_exclusive_scan(T x, T* total, T* s_wave)
{
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const T incl = wave_inclusive_scan(x);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWG / 64; ++w) {
        const T t = s_wave[w];
        if (w < wave) before += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + incl - x;
}

}  // namespace bfsmi
