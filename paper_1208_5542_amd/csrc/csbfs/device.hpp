// Wavefront helpers shared by the search kernels (not installed).
#pragma once

#include "common.hpp"

namespace csbfs {

__device__ __forceinline__ int wave_incl_scan_i32(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Owner lane of slot x: the largest lane L whose exclusive prefix excl[L] is
// at most x (excl non-decreasing over the lanes, excl[0] = 0).
__device__ __forceinline__ int owner_lane(int32_t excl, int32_t x) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int probe = lo + step;
        const int32_t ex = __shfl(excl, probe < 64 ? probe : 63, 64);
        if (probe < 64 && ex <= x) lo = probe;
    }
    return lo;
}

// Position of the r-th (0-based) set bit of w; w has more than r set bits.
__device__ __forceinline__ int select_bit(uint64_t w, int r) {
    int pos = 0;
    int c = __popc((uint32_t)w);
    if (r >= c) {
        r -= c;
        w >>= 32;
        pos += 32;
    }
    uint32_t x = (uint32_t)w;
    c = __popc(x & 0xFFFFu);
    if (r >= c) {
        r -= c;
        x >>= 16;
        pos += 16;
    }
    c = __popc(x & 0xFFu);
    if (r >= c) {
        r -= c;
        x >>= 8;
        pos += 8;
    }
    c = __popc(x & 0xFu);
    if (r >= c) {
        r -= c;
        x >>= 4;
        pos += 4;
    }
    c = __popc(x & 0x3u);
    if (r >= c) {
        r -= c;
        x >>= 2;
        pos += 2;
    }
    if (r >= (int)(x & 1u)) pos += 1;
    return pos;
}

__device__ __forceinline__ int64_t shfl64(int64_t v, int src) {
    const int32_t lo = __shfl((int32_t)(uint32_t)v, src, 64);
    const int32_t hi = __shfl((int32_t)(v >> 32), src, 64);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// Lane src of v (src wave-uniform) as a scalar, whatever the exec mask.
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v |= (uint64_t)shfl64((int64_t)v, (threadIdx.x & 63) ^ d);
    return v;
}

// Orders a wave's LDS stores before its later LDS loads by other lanes (and
// the loads before the next stores): LDS operations of one wave complete in
// order, so only the compiler must be kept from moving them.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds the workgroup's sum of v0 (and v1) to *d0 (and *d1) with one atomic
// per workgroup: every lane of a wave holds its wave's value. Device-scope
// atomics on one address are serialised at the memory side, so per-wave
// atomics on a shared counter cost far more than this LDS reduction. Must be
// reached by every thread of the workgroup.
template <int kWaves>
__device__ __forceinline__ void block_add(unsigned long long v0, unsigned long long *d0,
                                          unsigned long long v1 = 0, unsigned long long *d1 = nullptr) {
    __shared__ unsigned long long part[2][kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][w] = v0;
        part[1][w] = v1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s0 = 0, s1 = 0;
        for (int k = 0; k < kWaves; ++k) {
            s0 += part[0][k];
            s1 += part[1][k];
        }
        if (s0) atomicAdd(d0, s0);
        if (d1 && s1) atomicAdd(d1, s1);
    }
}

inline unsigned grid_for(int64_t items, int64_t per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace csbfs
