// Segmented LSD radix sort: every segment [seg_off[s], seg_off[s+1]) of a key
// array is sorted stably by key, one 8-bit digit per pass, least significant
// digit first.  Used for the local sort of the p segments (section 6, phase 1),
// for the per-bucket sort after the exchange (section 5) and for large probe
// sets.
//
// One pass = three launches:
//   count   -- workgroup (segment s, tile t) histograms the digit of its tile
//   scan    -- workgroup per segment turns the (tile, digit) counts into the
//              offset of every (digit, tile) run inside the segment
//   scatter -- workgroup (s, t) ranks its keys stably per digit with wave
//              ballots, stages the tile in LDS in digit order and writes each
//              digit run contiguously
// Tiles are kSortTile = 4096 keys; wave w of a tile owns the 1024 consecutive
// keys [w*1024, (w+1)*1024), read as 16 coalesced rows of 64 lanes.

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kWavesPerTile = kSortThreads / kWave;           // 4
constexpr int kKeysPerWave = kSortItems * kWave;              // 1024

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return (uint32_t)(k >> shift) & 0xFFu;
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(
    const K* __restrict__ keys, const uint64_t* __restrict__ seg_off, uint32_t tiles_per_seg,
    int shift, uint32_t* __restrict__ counts) {
    __shared__ uint32_t hist[256];
    const uint32_t seg = blockIdx.x / tiles_per_seg;
    const uint32_t tile = blockIdx.x % tiles_per_seg;
    hist[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b = seg_off[seg], e = seg_off[seg + 1];
    const uint64_t base = b + (uint64_t)tile * kSortTile;
    if (base < e) {
        const uint32_t n_tile = (uint32_t)min((uint64_t)kSortTile, e - base);
        const uint32_t w = threadIdx.x / kWave;
        const uint32_t lane = lane_id();
#pragma unroll 4
        for (int r = 0; r < kSortItems; ++r) {
            const uint32_t li = w * kKeysPerWave + r * kWave + lane;
            const bool valid = li < n_tile;
            const uint32_t d = valid ? digit_of(keys[base + li], shift) : 0u;
            const uint64_t live = __ballot(valid);
            if (live == 0) break;
            const uint64_t m = match_byte(d, live);
            if (valid && (m & lanes_below_mask()) == 0) atomicAdd(&hist[d], (uint32_t)__popcll(m));
        }
    }
    __syncthreads();
    counts[(uint64_t)blockIdx.x * 256 + threadIdx.x] = hist[threadIdx.x];
}

// counts[s][t][d] -> offset of the run of digit d from tile t inside segment s.
__global__ __launch_bounds__(256) void radix_scan_kernel(uint32_t* __restrict__ counts,
                                                         uint32_t tiles_per_seg) {
    __shared__ uint32_t scratch[256 / kWave];
    uint32_t* c = counts + (uint64_t)blockIdx.x * tiles_per_seg * 256;
    const uint32_t d = threadIdx.x;
    uint32_t tot = 0;
    for (uint32_t t = 0; t < tiles_per_seg; ++t) tot += c[t * 256 + d];
    uint32_t all;
    uint32_t run = block_exclusive_scan<uint32_t, 256>(tot, scratch, &all);
    for (uint32_t t = 0; t < tiles_per_seg; ++t) {
        const uint32_t x = c[t * 256 + d];
        c[t * 256 + d] = run;
        run += x;
    }
}

template <typename K, bool kPayload>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const K* __restrict__ kin, const uint64_t* __restrict__ vin, K* __restrict__ kout,
    uint64_t* __restrict__ vout, const uint64_t* __restrict__ seg_off, uint32_t tiles_per_seg,
    int shift, const uint32_t* __restrict__ counts) {
    __shared__ uint32_t whist[kWavesPerTile][256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t scratch[kSortThreads / kWave];
    __shared__ uint64_t stage[kSortTile];
    __shared__ uint8_t dstage[kSortTile];

    const uint32_t seg = blockIdx.x / tiles_per_seg;
    const uint32_t tile = blockIdx.x % tiles_per_seg;
    const uint64_t b = seg_off[seg], e = seg_off[seg + 1];
    const uint64_t base = b + (uint64_t)tile * kSortTile;
    if (base >= e) return;   // uniform over the workgroup
    const uint32_t n_tile = (uint32_t)min((uint64_t)kSortTile, e - base);
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();

    for (int i = threadIdx.x; i < kWavesPerTile * 256; i += kSortThreads) (&whist[0][0])[i] = 0;
    gofs[threadIdx.x] = counts[(uint64_t)blockIdx.x * 256 + threadIdx.x];
    __syncthreads();

    K key[kSortItems];
    uint32_t rank[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t li = w * kKeysPerWave + r * kWave + lane;
        const bool valid = li < n_tile;
        key[r] = valid ? kin[base + li] : (K)0;
        const uint32_t d = digit_of(key[r], shift);
        const uint64_t live = __ballot(valid);
        const uint64_t m = match_byte(d, live);
        const int leader = valid ? (int)(__ffsll((unsigned long long)m) - 1) : (int)lane;
        uint32_t old = 0;
        if (valid && (int)lane == leader) {
            old = whist[w][d];
            whist[w][d] = old + (uint32_t)__popcll(m);
        }
        old = __shfl(old, leader);
        rank[r] = old + (uint32_t)__popcll(m & lanes_below_mask());
    }
    __syncthreads();
    {
        const uint32_t d = threadIdx.x;
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < kWavesPerTile; ++ww) {
            const uint32_t t = whist[ww][d];
            whist[ww][d] = c;
            c += t;
        }
        uint32_t all;
        tstart[d] = block_exclusive_scan<uint32_t, kSortThreads>(c, scratch, &all);
    }
    __syncthreads();
    uint32_t pos[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t li = w * kKeysPerWave + r * kWave + lane;
        const uint32_t d = digit_of(key[r], shift);
        pos[r] = tstart[d] + whist[w][d] + rank[r];
        if (li < n_tile) {
            stage[pos[r]] = (uint64_t)key[r];
            dstage[pos[r]] = (uint8_t)d;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_tile; i += kSortThreads) {
        const uint32_t d = dstage[i];
        kout[b + gofs[d] + (i - tstart[d])] = (K)stage[i];
    }
    if constexpr (kPayload) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const uint32_t li = w * kKeysPerWave + r * kWave + lane;
            if (li < n_tile) stage[pos[r]] = vin[base + li];
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < n_tile; i += kSortThreads) {
            const uint32_t d = dstage[i];
            vout[b + gofs[d] + (i - tstart[d])] = stage[i];
        }
    }
}

template <typename K>
hipError_t run_sort(const SegSort& a, hipStream_t stream) {
    const uint32_t tps = (uint32_t)((a.max_seg_len + kSortTile - 1) / kSortTile);
    if (a.num_segs == 0 || tps == 0) return hipSuccess;
    const uint64_t grid = (uint64_t)a.num_segs * tps;
    const int passes = (a.end_bit - a.begin_bit + 7) / 8;
    const K* src = (const K*)a.keys_in;
    const uint64_t* vsrc = a.vals_in;
    const bool pay = a.vals_in != nullptr;
    for (int i = 0; i < passes; ++i) {
        const bool to_out = ((passes - 1 - i) % 2) == 0;
        K* dst = (K*)(to_out ? a.keys_out : a.keys_tmp);
        uint64_t* vdst = to_out ? a.vals_out : a.vals_tmp;
        const int shift = a.begin_bit + 8 * i;
        hipLaunchKernelGGL(radix_count_kernel<K>, dim3((unsigned)grid), dim3(kSortThreads), 0,
                           stream, src, a.seg_off, tps, shift, a.counts);
        hipLaunchKernelGGL(radix_scan_kernel, dim3(a.num_segs), dim3(256), 0, stream, a.counts,
                           tps);
        if (pay) {
            hipLaunchKernelGGL((radix_scatter_kernel<K, true>), dim3((unsigned)grid),
                               dim3(kSortThreads), 0, stream, src, vsrc, dst, vdst, a.seg_off, tps,
                               shift, a.counts);
        } else {
            hipLaunchKernelGGL((radix_scatter_kernel<K, false>), dim3((unsigned)grid),
                               dim3(kSortThreads), 0, stream, src, nullptr, dst, nullptr,
                               a.seg_off, tps, shift, a.counts);
        }
        src = dst;
        vsrc = vdst;
    }
    return hipGetLastError();
}

}  // namespace

uint64_t radix_count_words(uint32_t num_segs, uint64_t max_seg_len) {
    const uint64_t tps = (max_seg_len + kSortTile - 1) / kSortTile;
    return (uint64_t)num_segs * tps * 256;
}

hipError_t segmented_radix_sort(const SegSort& a, hipStream_t stream) {
    if (a.key_bytes == 4) return run_sort<uint32_t>(a, stream);
    return run_sort<uint64_t>(a, stream);
}

}  // namespace hss
