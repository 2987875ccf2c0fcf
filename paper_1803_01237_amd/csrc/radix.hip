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
//   scatter -- workgroup (s, t) ranks its keys per digit (stably with wave
//              ballots, or with LDS atomics when the order inside a run is
//              free), stages the tile in LDS in digit order and writes each
//              digit run contiguously
// Tiles are kSortTile = 4096 keys; wave w of a tile owns the 1024 consecutive
// keys [w*1024, (w+1)*1024), read as 16 coalesced rows of 64 lanes.

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kKeysPerWave = kSortItems * kWave;              // 1024
constexpr uint32_t kScatterTilesPerGroup = 1;                 // consecutive tiles per scatter workgroup
constexpr int kScatterThreads = 256;                           // threads of a scatter workgroup

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return (uint32_t)(k >> shift) & 0xFFu;
}

// Class of key k among the m splitters of a table T of kSplitSlots keys (the
// m splitters ascending, then all ones): with s the number of splitters below
// k, 2 s + 1 when k equals splitter s, else 2 s.  Binary lifting over the
// first kSplitSlots - 1 slots; the last slot is always padding.  A segment
// with no splitters keeps its digit.
__device__ __forceinline__ uint32_t split_class(const uint64_t* T, uint32_t m, uint64_t k) {
    uint32_t s = 0;
#pragma unroll
    for (uint32_t h = kSplitSlots / 2; h > 0; h >>= 1)
        if (T[s + h - 1] < k) s += h;
    return 2 * s + ((s < m && T[s] == k) ? 1u : 0u);
}

// A segment's splitter table into LDS (threads below kSplitSlots), with its
// splitter count.
__device__ __forceinline__ void load_splits(const TileMap& m, uint32_t seg, uint64_t* T, uint32_t* tm) {
    if (threadIdx.x < kSplitSlots) T[threadIdx.x] = m.splits[(uint64_t)seg * kSplitSlots + threadIdx.x];
    if (threadIdx.x == 0) *tm = m.n_splits[seg];
}

// Key range [base, stop) of workgroup tile `bid`; false when it is empty.
__device__ __forceinline__ bool tile_range(const TileMap& m, uint32_t bid, uint64_t* base,
                                           uint64_t* stop, uint32_t* seg) {
    uint32_t s, t;
    if (m.tile_seg) {
        s = m.tile_seg[bid];
        t = bid - m.tile0[s];
    } else {
        s = bid / m.tps;
        t = bid % m.tps;
    }
    const uint64_t b = m.beg[s], e = m.end[s];
    *seg = s;
    *base = b + (uint64_t)t * kSortTile;
    *stop = e;
    return *base < e;
}

// First key of the tile starting at position `base` of segment `seg`.
template <typename K>
__device__ __forceinline__ const K* tile_source(const TileMap& m, const K* in, uint32_t seg,
                                                uint64_t base) {
    if (m.src) return (const K*)(uintptr_t)m.src[seg] + (base - m.beg[seg]);
    return in + base;
}

__device__ __forceinline__ const uint64_t* tile_vsource(const TileMap& m, const uint64_t* in,
                                                        uint32_t seg, uint64_t base) {
    if (m.vsrc) return (const uint64_t*)(uintptr_t)m.vsrc[seg] + (base - m.beg[seg]);
    return in + base;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// kMask: also the AND and OR of every key - base of the segment (which bits
// vary inside it), one pair of atomics per tile.  kSplit: the "digit" of a
// key is its class among the segment's splitters.
template <typename K, bool kMask, bool kSplit>
__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(const K* __restrict__ keys,
                                                                   TileMap m, int shift,
                                                                   const uint8_t* __restrict__ seg_shift,
                                                                   uint32_t* __restrict__ counts,
                                                                   uint64_t* __restrict__ and_mask,
                                                                   uint64_t* __restrict__ or_mask) {
    static_assert(kSortThreads >= (int)kSplitSlots, "one thread per splitter slot");
    __shared__ uint32_t hist[256];
    __shared__ uint64_t wmask[kMask ? kSortThreads / kWave : 1][2];
    __shared__ uint64_t T[kSplit ? kSplitSlots : 1];
    __shared__ uint32_t tm;
    hist[threadIdx.x] = 0;
    bool in_seg = false;
    uint32_t mseg = 0;
    uint64_t base, e;
    uint32_t seg;
    const bool has = tile_range(m, blockIdx.x, &base, &e, &seg);
    if constexpr (kSplit) {
        if (has) load_splits(m, seg, T, &tm);
    }
    __syncthreads();
    if (has) {
        in_seg = true;
        mseg = seg;
        if (seg_shift) shift = seg_shift[seg];
        const K kb = m.base ? (K)m.base[seg] : (K)0;
        const uint32_t n_tile = (uint32_t)min((uint64_t)kSortTile, e - base);
        const uint32_t w = threadIdx.x / kWave;
        const uint32_t lane = lane_id();
        const K* src = tile_source(m, keys, seg, base);
        // all loads of the tile in flight before any counting
        K kr[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const uint32_t li = w * kKeysPerWave + r * kWave + lane;
            kr[r] = li < n_tile ? ld_stream(src + li) : (K)0;
        }
        // a class: every row's search in flight together
        uint32_t dg[kSplit ? kSortItems : 1];
        if constexpr (kSplit) {
            const uint32_t nsp = tm;
#pragma unroll
            for (int r = 0; r < kSortItems; ++r)
                dg[r] = nsp ? split_class(T, nsp, (uint64_t)kr[r]) : digit_of((K)(kr[r] - kb), shift);
        }
        auto dk = [&](int r) -> uint32_t {
            if constexpr (kSplit) return dg[r];
            else return digit_of((K)(kr[r] - kb), shift);
        };
        // skewed inputs: the lanes holding the wave's current dominant digit
        // add with one atomic (many lanes on one LDS counter would take turns)
        uint32_t dom = dk(0);
        dom = (uint32_t)__shfl((int)dom, 0);
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const uint32_t li = w * kKeysPerWave + r * kWave + lane;
            const bool valid = li < n_tile;
            const uint32_t d = dk(r);
            const uint64_t md = __ballot(valid && d == dom);
            const uint32_t nd = (uint32_t)__popcll(md);
            if (nd && (int)lane == __ffsll((unsigned long long)md) - 1) atomicAdd(&hist[dom], nd);
            if (valid && d != dom) atomicAdd(&hist[d], 1u);
            // the digit stays dominant while it holds a quarter of a row
            if (nd < kWave / 4) dom = (uint32_t)__shfl((int)d, 0);
        }
        if constexpr (kMask) {
            uint64_t am = ~0ull, om = 0;
#pragma unroll
            for (int r = 0; r < kSortItems; ++r) {
                const uint32_t li = w * kKeysPerWave + r * kWave + lane;
                if (li < n_tile) {
                    const uint64_t x = (uint64_t)(K)(kr[r] - kb);
                    am &= x;
                    om |= x;
                }
            }
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) {
                am &= shfl_xor_u64(am, o);
                om |= shfl_xor_u64(om, o);
            }
            if (lane == 0) {
                wmask[w][0] = am;
                wmask[w][1] = om;
            }
        }
    }
    __syncthreads();
    counts[(uint64_t)blockIdx.x * 256 + threadIdx.x] = hist[threadIdx.x];
    if constexpr (kMask) {
        if (in_seg && threadIdx.x == 0) {
            uint64_t am = ~0ull, om = 0;
#pragma unroll
            for (int q = 0; q < kSortThreads / kWave; ++q) {
                am &= wmask[q][0];
                om |= wmask[q][1];
            }
            atomicAnd((unsigned long long*)&and_mask[mseg], (unsigned long long)am);
            atomicOr((unsigned long long*)&or_mask[mseg], (unsigned long long)om);
        }
    }
}

// counts[tile][d] of one segment's tiles -> offset of the run of digit d from
// that tile inside the segment.  Optionally records, per (segment, digit), the
// start and length of the digit's run: the sub-buckets of an MSD pass.
__global__ __launch_bounds__(256) void radix_scan_kernel(uint32_t* __restrict__ counts, TileMap m,
                                                         uint64_t* __restrict__ sb_start,
                                                         uint32_t* __restrict__ sb_len) {
    __shared__ uint32_t scratch[256 / kWave];
    const uint32_t s = blockIdx.x;
    uint32_t t0, nt;
    if (m.tile_seg) {
        t0 = m.tile0[s];
        nt = m.tile0[s + 1] - t0;
    } else {
        t0 = s * m.tps;
        nt = m.tps;
    }
    uint32_t* c = counts + (uint64_t)t0 * 256;
    const uint32_t d = threadIdx.x;
    uint32_t tot = 0;
    for (uint32_t t = 0; t < nt; ++t) tot += c[t * 256 + d];
    uint32_t all;
    uint32_t run = block_exclusive_scan<uint32_t, 256>(tot, scratch, &all);
    if (sb_start) {
        sb_start[(uint64_t)s * 256 + d] = m.beg[s] + run;
        sb_len[(uint64_t)s * 256 + d] = tot;
    }
    for (uint32_t t = 0; t < nt; ++t) {
        const uint32_t x = c[t * 256 + d];
        c[t * 256 + d] = run;
        run += x;
    }
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  The
// tile of workgroup b is chosen so that every XCD walks one contiguous range
// of tiles in order: neighbouring tiles of a segment then write the two parts
// of a shared cache line through the same L2.  A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    constexpr uint32_t kXcds = 8;
    const uint32_t q = n / kXcds, r = n % kXcds;
    const uint32_t x = b % kXcds, l = b / kXcds;
    return x * q + min(x, r) + l;
}

// Placement of one tile by digit; the tile is staged in LDS in digit order and
// written out digit run by digit run.  kStable: each wave ranks its keys among
// equal digits with ballots (a wave owns a contiguous quarter of the tile,
// rows of 64 keys in order) and per-wave digit counts give the offsets, so
// equal digits keep their input order.  Otherwise one LDS atomic per key
// hands out the slots of its digit in arbitrary order.  kSplit: the digit of
// a key is its class among the segment's splitters.
template <typename K, bool kPayload, bool kStable, bool kSplit>
__global__ __launch_bounds__(kScatterThreads) void radix_scatter_kernel(
    const K* __restrict__ kin, const uint64_t* __restrict__ vin, K* __restrict__ kout,
    uint64_t* __restrict__ vout, TileMap m, int shift0, const uint8_t* __restrict__ seg_shift,
    const uint32_t* __restrict__ counts, uint32_t num_tiles) {
    static_assert(kStable || !kPayload, "a payload needs the stable placement");
    constexpr int kWv = kScatterThreads / kWave;          // waves per tile
    constexpr int kIt = kSortTile / kScatterThreads;      // keys per thread
    constexpr int kKpw = kIt * kWave;                     // keys per wave
    static_assert(kScatterThreads >= 256 && kIt * kScatterThreads == kSortTile, "tile shape");
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t whist[kStable ? kWv : 1][256];
    __shared__ uint32_t scratch[kScatterThreads / kWave];
    __shared__ uint64_t stage[kSortTile];
    __shared__ uint16_t sidx[kPayload ? kSortTile : 1];   // input index of each staged key
    __shared__ uint64_t T[kSplit ? kSplitSlots : 1];
    __shared__ uint32_t tm;
    __shared__ uint8_t sdig[kSplit ? kSortTile : 1];      // class of each staged key

    const uint32_t w = threadIdx.x / kWave;
    const uint32_t lane = lane_id();
    const bool digit_thread = threadIdx.x < 256;   // one thread per digit for the tables
    for (uint32_t sub = 0; sub < kScatterTilesPerGroup; ++sub) {
        const uint32_t tile = xcd_contiguous(blockIdx.x, gridDim.x) * kScatterTilesPerGroup + sub;
        if (tile >= num_tiles) break;   // uniform over the workgroup
        uint64_t base, e;
        uint32_t seg;
        if (!tile_range(m, tile, &base, &e, &seg)) continue;   // uniform
        if (m.skip && m.skip[seg]) continue;                   // uniform
        const int shift = seg_shift ? (int)seg_shift[seg] : shift0;
        const K kb = m.base ? (K)m.base[seg] : (K)0;
        const uint64_t b = m.beg[seg];
        const uint32_t n_tile = (uint32_t)min((uint64_t)kSortTile, e - base);

        if (sub) __syncthreads();   // the previous tile is done with the LDS
        for (int i = threadIdx.x; i < (kStable ? kWv : 1) * 256; i += kScatterThreads) (&whist[0][0])[i] = 0;
        if (digit_thread) gofs[threadIdx.x] = counts[(uint64_t)tile * 256 + threadIdx.x];
        if constexpr (kSplit) load_splits(m, seg, T, &tm);
        __syncthreads();
        auto dig = [&](K k) -> uint32_t {
            if constexpr (kSplit) return tm ? split_class(T, tm, (uint64_t)k) : digit_of((K)(k - kb), shift);
            else return digit_of((K)(k - kb), shift);
        };

        const K* src = tile_source(m, kin, seg, base);
        K key[kIt];
        uint32_t rank[kIt];
#pragma unroll
        for (int r = 0; r < kIt; ++r) {
            const uint32_t li = w * kKpw + r * kWave + lane;
            key[r] = li < n_tile ? ld_stream(src + li) : (K)0;
        }
        // a class is found once per key (all rows' searches in flight
        // together) and kept beside the staged key; a digit is recomputed
        uint32_t dg[kSplit ? kIt : 1];
        if constexpr (kSplit) {
#pragma unroll
            for (int r = 0; r < kIt; ++r) dg[r] = dig(key[r]);
        }
        auto dk = [&](int r) -> uint32_t {
            if constexpr (kSplit) return dg[r];
            else return dig(key[r]);
        };
        if constexpr (kStable) {
#pragma unroll
            for (int r = 0; r < kIt; ++r) {
                const uint32_t li = w * kKpw + r * kWave + lane;
                const bool valid = li < n_tile;
                const uint32_t d = dk(r);
                const uint64_t live = __ballot(valid);
                const uint64_t mm = match_byte(d, live);
                const int leader = valid ? (int)(__ffsll((unsigned long long)mm) - 1) : (int)lane;
                uint32_t old = 0;
                if (valid && (int)lane == leader) {
                    old = whist[w][d];
                    whist[w][d] = old + (uint32_t)__popcll(mm);
                }
                old = __shfl(old, leader);
                rank[r] = old + (uint32_t)__popcll(mm & lanes_below_mask());
            }
            __syncthreads();
            {
                const uint32_t d = threadIdx.x;
                uint32_t c = 0;
                if (digit_thread) {
#pragma unroll
                    for (int ww = 0; ww < kWv; ++ww) {
                        const uint32_t t = whist[ww][d];
                        whist[ww][d] = c;
                        c += t;
                    }
                }
                uint32_t all;
                const uint32_t st = block_exclusive_scan<uint32_t, kScatterThreads>(c, scratch, &all);
                if (digit_thread) tstart[d] = st;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kIt; ++r) {
                const uint32_t li = w * kKpw + r * kWave + lane;
                if (li < n_tile) {
                    const uint32_t d = dk(r);
                    const uint32_t pos = tstart[d] + whist[w][d] + rank[r];
                    stage[pos] = (uint64_t)key[r];
                    if constexpr (kPayload) sidx[pos] = (uint16_t)li;
                    if constexpr (kSplit) sdig[pos] = (uint8_t)d;
                }
            }
        } else {
            uint32_t* hist = &whist[0][0];   // one tile-wide count per digit
            // the lanes holding the wave's current dominant digit take their
            // slots with one atomic (skewed inputs), the others one each
            uint32_t dom = dk(0);
            dom = (uint32_t)__shfl((int)dom, 0);
#pragma unroll
            for (int r = 0; r < kIt; ++r) {
                const uint32_t li = w * kKpw + r * kWave + lane;
                const bool valid = li < n_tile;
                const uint32_t d = dk(r);
                const uint64_t md = __ballot(valid && d == dom);
                const uint32_t nd = (uint32_t)__popcll(md);
                uint32_t b0 = 0;
                if (nd) {   // uniform
                    const int leader = __ffsll((unsigned long long)md) - 1;
                    if ((int)lane == leader) b0 = atomicAdd(&hist[dom], nd);
                    b0 = (uint32_t)__shfl((int)b0, leader);
                }
                if (valid) rank[r] = d == dom ? b0 + (uint32_t)__popcll(md & lanes_below_mask()) : atomicAdd(&hist[d], 1u);
                if (nd < kWave / 4) dom = (uint32_t)__shfl((int)d, 0);
            }
            __syncthreads();
            uint32_t all;
            const uint32_t st = block_exclusive_scan<uint32_t, kScatterThreads>(
                digit_thread ? hist[threadIdx.x] : 0u, scratch, &all);
            if (digit_thread) tstart[threadIdx.x] = st;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kIt; ++r) {
                const uint32_t li = w * kKpw + r * kWave + lane;
                if (li < n_tile) {
                    const uint32_t d = dk(r);
                    stage[tstart[d] + rank[r]] = (uint64_t)key[r];
                    if constexpr (kSplit) sdig[tstart[d] + rank[r]] = (uint8_t)d;
                }
            }
        }
        __syncthreads();
        const uint64_t* vsrc = kPayload ? tile_vsource(m, vin, seg, base) : nullptr;
        // the segment's output: at its own position of the pass output, or
        // at its listed destination
        K* ko = m.dst ? (K*)(uintptr_t)m.dst[seg] : kout + b;
        uint64_t* vo = kPayload ? (m.vdst ? (uint64_t*)(uintptr_t)m.vdst[seg] : vout + b) : nullptr;
        if constexpr (kPayload) {
            // every payload word of the thread's outputs is gathered (from
            // the tile's input, which the L2 holds) before the first store
            uint64_t pv[kIt];
#pragma unroll
            for (int r = 0; r < kIt; ++r) {
                const uint32_t i = r * kScatterThreads + threadIdx.x;
                pv[r] = i < n_tile ? as_global(vsrc)[sidx[i]] : 0;
            }
#pragma unroll
            for (int r = 0; r < kIt; ++r) {
                const uint32_t i = r * kScatterThreads + threadIdx.x;
                if (i < n_tile) {
                    const K k = (K)stage[i];
                    uint32_t d;
                    if constexpr (kSplit) d = sdig[i];
                    else d = dig(k);
                    const uint64_t dst = gofs[d] + (i - tstart[d]);
                    as_global(ko)[dst] = k;
                    as_global(vo)[dst] = pv[r];
                }
            }
        } else {
            for (uint32_t i = threadIdx.x; i < n_tile; i += kScatterThreads) {
                const K k = (K)stage[i];
                uint32_t d;
                if constexpr (kSplit) d = sdig[i];
                else d = dig(k);
                const uint64_t dst = gofs[d] + (i - tstart[d]);
                // plain stores: a digit run covers parts of cache lines, which
                // the L2 merges before they go out
                as_global(ko)[dst] = k;
            }
        }
    }
}

// algorithmic bytes: the keys (and payload) are read by the count pass, read
// and written by the scatter pass; the count table is written by the count
// pass, read and written by the scan, read by the scatter pass
template <typename K>
hipError_t count_scan_impl(const RadixPass& a, hipStream_t stream) {
    if (a.num_segs == 0 || a.num_tiles == 0) return hipSuccess;
    Profiler dummy;
    Profiler& prof = a.prof ? *a.prof : dummy;
    const uint64_t table = (uint64_t)a.num_tiles * 256ull * 4ull;
    const dim3 grid(a.num_tiles), block(kSortThreads);
    prof.begin(stream);
    if (a.counted) {
        // counted where the keys were written
    } else if (a.map.splits)   // a splitter level (its masks are always taken)
        hipLaunchKernelGGL((radix_count_kernel<K, true, true>), grid, block, 0, stream, (const K*)a.keys_in,
                           a.map, a.shift, a.seg_shift, a.counts, a.and_mask, a.or_mask);
    else if (a.and_mask)
        hipLaunchKernelGGL((radix_count_kernel<K, true, false>), grid, block, 0, stream, (const K*)a.keys_in,
                           a.map, a.shift, a.seg_shift, a.counts, a.and_mask, a.or_mask);
    else
        hipLaunchKernelGGL((radix_count_kernel<K, false, false>), grid, block, 0, stream, (const K*)a.keys_in,
                           a.map, a.shift, a.seg_shift, a.counts, nullptr, nullptr);
    prof.end(kProfRadixCount, stream, a.total_len * sizeof(K) + table);
    prof.begin(stream);
    hipLaunchKernelGGL(radix_scan_kernel, dim3(a.num_segs), dim3(256), 0, stream, a.counts, a.map,
                       a.sb_start, a.sb_len);
    prof.end(kProfRadixScan, stream, 2 * table);
    return hipGetLastError();
}

template <typename K>
hipError_t scatter_impl(const RadixPass& a, hipStream_t stream) {
    if (a.num_segs == 0 || a.num_tiles == 0) return hipSuccess;
    Profiler dummy;
    Profiler& prof = a.prof ? *a.prof : dummy;
    const bool pay = a.vals_in != nullptr || a.has_payload;
    const uint64_t table = (uint64_t)a.num_tiles * 256ull * 4ull;
    prof.begin(stream);
    const dim3 sgrid((a.num_tiles + kScatterTilesPerGroup - 1) / kScatterTilesPerGroup);
    const dim3 sblock(kScatterThreads);
    const bool split = a.map.splits != nullptr;
    if (pay) {
        if (split)
            hipLaunchKernelGGL((radix_scatter_kernel<K, true, true, true>), sgrid, sblock, 0, stream,
                               (const K*)a.keys_in, a.vals_in, (K*)a.keys_out, a.vals_out, a.map,
                               a.shift, a.seg_shift, a.counts, a.num_tiles);
        else
            hipLaunchKernelGGL((radix_scatter_kernel<K, true, true, false>), sgrid, sblock, 0, stream,
                               (const K*)a.keys_in, a.vals_in, (K*)a.keys_out, a.vals_out, a.map,
                               a.shift, a.seg_shift, a.counts, a.num_tiles);
    } else if (a.any_order) {
        if (split)
            hipLaunchKernelGGL((radix_scatter_kernel<K, false, false, true>), sgrid, sblock, 0, stream,
                               (const K*)a.keys_in, nullptr, (K*)a.keys_out, nullptr, a.map, a.shift,
                               a.seg_shift, a.counts, a.num_tiles);
        else
            hipLaunchKernelGGL((radix_scatter_kernel<K, false, false, false>), sgrid, sblock, 0, stream,
                               (const K*)a.keys_in, nullptr, (K*)a.keys_out, nullptr, a.map, a.shift,
                               a.seg_shift, a.counts, a.num_tiles);
    } else {
        if (split)
            hipLaunchKernelGGL((radix_scatter_kernel<K, false, true, true>), sgrid, sblock, 0, stream,
                               (const K*)a.keys_in, nullptr, (K*)a.keys_out, nullptr, a.map, a.shift,
                               a.seg_shift, a.counts, a.num_tiles);
        else
            hipLaunchKernelGGL((radix_scatter_kernel<K, false, true, false>), sgrid, sblock, 0, stream,
                               (const K*)a.keys_in, nullptr, (K*)a.keys_out, nullptr, a.map, a.shift,
                               a.seg_shift, a.counts, a.num_tiles);
    }
    prof.end(kProfRadixScatter, stream,
             a.total_len * 2 * (sizeof(K) + (pay ? 8 : 0)) + table);
    return hipGetLastError();
}

}  // namespace

hipError_t radix_count_scan(const RadixPass& a, hipStream_t stream) {
    if (a.key_bytes == 4) return count_scan_impl<uint32_t>(a, stream);
    return count_scan_impl<uint64_t>(a, stream);
}

hipError_t radix_scatter(const RadixPass& a, hipStream_t stream) {
    if (a.key_bytes == 4) return scatter_impl<uint32_t>(a, stream);
    return scatter_impl<uint64_t>(a, stream);
}

hipError_t radix_pass(const RadixPass& a, hipStream_t stream) {
    const hipError_t e = radix_count_scan(a, stream);
    if (e != hipSuccess) return e;
    return radix_scatter(a, stream);
}

uint64_t radix_count_words(uint32_t num_segs, uint64_t max_seg_len) {
    const uint64_t tps = (max_seg_len + kSortTile - 1) / kSortTile;
    return (uint64_t)num_segs * tps * 256;
}

// Plain LSD over contiguous segments: ceil((end_bit - begin_bit) / 8) passes,
// the last one into keys_out.
hipError_t segmented_radix_sort(const SegSort& a, hipStream_t stream) {
    const uint32_t tps = (uint32_t)((a.max_seg_len + kSortTile - 1) / kSortTile);
    if (a.num_segs == 0 || tps == 0) return hipSuccess;
    const int passes = (a.end_bit - a.begin_bit + 7) / 8;
    RadixPass ps;
    ps.key_bytes = a.key_bytes;
    ps.map.beg = a.seg_off;
    ps.map.end = a.seg_off + 1;
    ps.map.tps = tps;
    ps.num_segs = a.num_segs;
    ps.num_tiles = a.num_segs * tps;
    ps.counts = a.counts;
    ps.total_len = a.total_len;
    ps.prof = a.prof;
    const void* src = a.keys_in;
    const uint64_t* vsrc = a.vals_in;
    for (int i = 0; i < passes; ++i) {
        const bool to_out = ((passes - 1 - i) % 2) == 0;
        ps.keys_in = src;
        ps.vals_in = vsrc;
        ps.keys_out = to_out ? a.keys_out : a.keys_tmp;
        ps.vals_out = to_out ? a.vals_out : a.vals_tmp;
        ps.shift = a.begin_bit + 8 * i;
        hipError_t e = radix_pass(ps, stream);
        if (e != hipSuccess) return e;
        src = ps.keys_out;
        vsrc = ps.vals_out;
    }
    return hipSuccess;
}

}  // namespace hss
