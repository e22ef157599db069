// Shared device helpers for the gfx950 (CDNA4, wave64) triangle-counting library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcx {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
// Uniform across the wave; readfirstlane lets the compiler keep values derived
// from it in scalar registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)); }

// Bit mask of the lanes below the calling lane.
__device__ __forceinline__ uint64_t lanes_below() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (WAVE - l));
}

// Lanes of the wave whose 8-bit digit equals this lane's, restricted to `active`.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t active) {
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, WAVE);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), o, WAVE);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Inclusive scan across the wave (Hillis-Steele with shuffles).
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const T t = __shfl_up(v, o, WAVE);
        if (l >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over a block of NT threads.
// `scratch` must hold NT / WAVE elements; the call contains barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* scratch, T* total = nullptr) {
    const T inc = wave_inclusive_scan(v);
    const int w = wave_id();
    if (lane_id() == WAVE - 1) scratch[w] = inc;
    __syncthreads();
    T wave_base = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i) {
        const T s = scratch[i];
        if (i < w) wave_base += s;
        all += s;
    }
    if (total) *total = all;
    __syncthreads();
    return wave_base + inc - v;
}

// First-pass digit counts of a radix sort, gathered by the kernel that writes
// the keys: a block of 256 threads writes tile t (the sort's tile of consecutive keys)
// and adds each key's first digit here; flush() stores the tile's column of
// the count table (256 digit rows) and clears the counters.
struct TileCounts {
    uint32_t w[4][256];   // one histogram per wave (256 threads)
    __device__ void clear() {
        for (int i = threadIdx.x; i < 4 * 256; i += 256) (&w[0][0])[i] = 0;
    }
    __device__ void add(uint32_t digit) { atomicAdd(&w[threadIdx.x >> 6][digit], 1u); }
    // Whole block; barriers.
    __device__ void flush(uint32_t* counts, uint32_t ntiles, uint32_t tile) {
        __syncthreads();
        const uint32_t d = threadIdx.x;
        counts[(size_t)d * ntiles + tile] = w[0][d] + w[1][d] + w[2][d] + w[3][d];
        w[0][d] = w[1][d] = w[2][d] = w[3][d] = 0;
        __syncthreads();
    }
};

// Ceiling of log2 for x >= 1 (number of bits needed to hold values < x).
__host__ __device__ __forceinline__ int bits_for(uint64_t x) {
    int b = 0;
    while (b < 64 && (1ull << b) < x) ++b;
    return b;
}

// floor(log2 x) for x >= 1.
__device__ __forceinline__ int floor_log2(uint32_t x) { return 31 - __clz(x); }

}  // namespace tcx
