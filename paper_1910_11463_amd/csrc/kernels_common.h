// Device-side helpers shared by the HIP kernels (wave64 reductions and scans,
// the SplitMix64 generator).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pair {

__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ __forceinline__ int wave_inclusive_scan_int(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Sum over groups of G consecutive lanes (G a power of two <= 64); every lane of
// the group receives the group total.  The reduction tree is fixed, so the
// result is bitwise reproducible.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <int G>
__device__ __forceinline__ int group_sum_int(int v) {
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <int G>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
    for (int d = G / 2; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}

// Append to a global list with one atomic per block: every thread of the
// one-dimensional NT-thread block must call this.  Returns the slot of the
// calling thread, or -1.  The order of entries across blocks is not fixed.
template <int NT>
__device__ __forceinline__ int block_append(bool pred, int* counter) {
    __shared__ int s_cnt[NT / 64];
    __shared__ int s_base;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t m = __ballot(pred);
    if (lane == 0) s_cnt[wid] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < NT / 64; ++w) {
            const int t = s_cnt[w];
            s_cnt[w] = tot;
            tot += t;
        }
        s_base = tot > 0 ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    const int slot = s_base + s_cnt[wid] + __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();   // the next call may overwrite s_cnt / s_base
    return pred ? slot : -1;
}

// Reserves c consecutive slots per thread in a global list (block-wide
// exclusive scan of c, one atomicAdd on `counter` per block); returns the
// thread's first slot.  Every thread of the NT-thread block must call it.
template <int NT>
__device__ __forceinline__ int block_reserve(int c, int* counter) {
    __shared__ int s_w[NT / 64];
    __shared__ int s_base;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < NT / 64; ++w) {
            const int t = s_w[w];
            s_w[w] = tot;
            tot += t;
        }
        s_base = tot > 0 ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    const int slot = s_base + s_w[wid] + x - c;
    __syncthreads();   // the next call may overwrite s_w / s_base
    return slot;
}

// SplitMix64 (Steele, Lea & Flood 2014): add the golden-ratio increment, then
// the variant-13 finaliser.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 53-bit random integer of local row i on a level (PMIS measure tie-breaker).
__device__ __forceinline__ uint64_t pmis_rand(uint64_t seed, int level, int64_t i) {
    uint64_t key = (seed << 40) + (static_cast<uint64_t>(level) << 32) + static_cast<uint64_t>(i);
    return splitmix64(key) >> 11;
}

}  // namespace pair
