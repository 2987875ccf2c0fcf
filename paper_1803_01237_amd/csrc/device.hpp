// Device-side building blocks shared by the HSS kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hss {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32 with 10 rounds (Salmon et al., SC'11).
// State is the 128-bit counter; the 64-bit key is bumped by the golden-ratio
// and sqrt(3)-1 Weyl increments after every round but the last.
// ---------------------------------------------------------------------------
struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply gives both halves of each product
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        c0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        c2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// The 4 sampling words of tag block b = g >> 2 in round j: counter
// (b_lo, b_hi, j, 0), key = seed.
__device__ __forceinline__ Philox4 sample_block(uint64_t seed, uint64_t block, uint32_t round) {
    return philox10((uint32_t)block, (uint32_t)(block >> 32), round, 0u, (uint32_t)seed,
                    (uint32_t)(seed >> 32));
}

// ---------------------------------------------------------------------------
// Wave helpers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Global-memory view of a pointer.  A pointer taken from a table of device
// addresses, or chosen between two buffers, is generic to the compiler, which
// then emits flat accesses; a flat load also counts against the LDS wait
// counter, so every wait for an LDS result waits for the key loads as well.
template <typename T>
using global_ptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ global_ptr<T> as_global(const T* p) {
    return (global_ptr<T>)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Streaming accesses: loads and stores of data touched once per pass, issued
// with the non-temporal hint so that they do not displace what is reused.
// Only for accesses that take whole cache lines at once (a tile read in
// rows, a sub-bucket written by one workgroup): a line consumed piece by
// piece (digit runs, short pieces, gathers inside a tile) is fetched or
// written again for every piece when it is not kept.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(as_global(p));
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    __builtin_nontemporal_store(v, as_global(p));
}

__device__ __forceinline__ uint64_t lanes_below_mask() {
    return (1ull << lane_id()) - 1ull;   // lane 0 -> 0
}

// Lanes of the wave whose 8-bit value equals this lane's, among `live` lanes.
__device__ __forceinline__ uint64_t match_byte(uint32_t d, uint64_t live) {
    uint64_t m = live;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t set = __ballot(bit);
        m &= bit ? set : ~set;
    }
    return m;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = __shfl((uint32_t)v, src);
    uint32_t hi = __shfl((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        if constexpr (sizeof(T) == 8) {
            v += (T)shfl_u64((uint64_t)v, (int)(lane_id() ^ off));
        } else {
            v += (T)__shfl((uint32_t)v, (int)(lane_id() ^ off));
        }
    }
    return v;
}

// Block-wide sum; `scratch` holds one slot per wave.  All threads get the sum.
template <typename T, int kThreads>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
    constexpr int kWaves = kThreads / kWave;
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    T t = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += scratch[i];
    __syncthreads();
    return t;
}

// Inclusive prefix sum inside a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T o;
        if constexpr (sizeof(T) == 8) {
            o = (T)shfl_u64((uint64_t)v, (int)(lane >= (uint32_t)off ? lane - off : lane));
        } else {
            o = (T)__shfl((uint32_t)v, (int)(lane >= (uint32_t)off ? lane - off : lane));
        }
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}

// Block exclusive scan of one value per thread; returns the exclusive prefix
// and writes the block total to *total.  `scratch` holds one slot per wave.
template <typename T, int kThreads>
__device__ __forceinline__ T block_exclusive_scan(T v, T* scratch, T* total) {
    constexpr int kWaves = kThreads / kWave;
    const int w = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane_id() == kWave - 1) scratch[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        const T s = scratch[i];
        if (i < w) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Number of elements of the sorted run a[0, len) that precede probe key `k`
// when equal keys precede (upper bound, `equal_before`) or follow (lower bound).
template <typename K>
__device__ __forceinline__ uint64_t count_before(const K* __restrict__ a, uint64_t lo, uint64_t hi,
                                                 K k, bool equal_before) {
    // invariant: answer in [lo, hi]
    while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        const K x = a[mid];
        const bool go_right = equal_before ? (x <= k) : (x < k);
        if (go_right) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace hss
