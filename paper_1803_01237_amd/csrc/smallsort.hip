// Segmented stable sort by MSD splitting plus on-chip finishing.
//
//   1. one counting pass on the top 8 bits of the key (count / scan / scatter
//      of radix.hip) moves every segment into 256 sub-buckets, in the
//      temporary buffer; the scan records each sub-bucket's start and length
//   2. one workgroup per sub-bucket of at most kCap keys sorts it on chip by
//      the remaining bits and writes it to the output:
//        - the keys are dropped into groups by the next 8 bits in LDS, and
//          when no group exceeds kGroupMax keys, each key's place inside its
//          group is counted directly (keys smaller, or equal and earlier);
//        - otherwise the sub-bucket is listed for a second kernel that runs
//          LSD counting passes in LDS over the remaining digits, skipping
//          digits on which all its keys agree
//   3. sub-buckets larger than kCap are collected into a compact list and go
//      through LSD counting passes in HBM (radix.hip, list mode)
// With a payload every step is stable, so equal keys keep their input order;
// keys alone may swap places with equal keys, which leaves the output the same.

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kT = 256;
constexpr int kW = kT / kWave;               // waves per workgroup
constexpr int kCapSmall = 2048;              // largest sub-bucket sorted in LDS (local sort)
static_assert(kDirectSegMax <= (uint32_t)kCapSmall, "direct segments fit the small sort");
constexpr int kCapLarge = 4096;              // same for the bucket sort
constexpr int kCap = kCapLarge;              // the LDS-LSD kernel handles any of them
constexpr int kRows = kCap / kT;             // rows of 64 keys per wave at kCap
constexpr uint32_t kGroupMax = 32;           // largest group ranked by direct counting
constexpr int kGroupBits = 9;                // bits of the second-level groups of the fast path

template <typename K>
__device__ __forceinline__ uint32_t dig(K k, int shift) {
    return (uint32_t)(k >> shift) & 0xFFu;
}

// Records the key written at output position o of segment seg when o falls
// on a fence position of that segment.
// Where the fences of one segment go: fence f of the segment is the key at
// position org + f * kFenceStride; dst is null when no fences are kept.
struct FenceSink {
    uint64_t* dst;
    uint64_t org;
};

__device__ __forceinline__ FenceSink fence_sink(const Fences& f, uint32_t seg) {
    if (!f.key) return FenceSink{nullptr, 0};
    return FenceSink{f.key + f.base[seg], f.seg_off[seg]};
}

__device__ __forceinline__ void put_fence(const FenceSink& fs, uint64_t o, uint64_t key) {
    const uint64_t rel = o - fs.org;
    if ((rel & (kFenceStride - 1)) == 0) fs.dst[rel / kFenceStride] = key;
}

// Stable counting pass in LDS: the n keys of `sk` (with indices `si`, or the
// identity when null) are placed by the digit of key - kbase at `shift` into
// `dk` / `di`.
// Leaves the digit starts in start[0..256] and the largest digit count in
// *max_count.  Wave w handles the keys [w*cw, (w+1)*cw) in rows of 64.
template <typename K>
__device__ void lds_pass(const K* sk, const uint16_t* si, K* dk, uint16_t* di, uint32_t n,
                         int shift, K kbase, uint32_t (*whist)[256], uint32_t* start,
                         uint32_t* scratch, uint32_t* max_count) {
    const uint32_t cw = ((n + kW * kWave - 1) / (kW * kWave)) * kWave;
    const uint32_t rows = cw / kWave;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    for (int i = threadIdx.x; i < kW * 256; i += kT) (&whist[0][0])[i] = 0;
    if (threadIdx.x == 0) *max_count = 0;
    __syncthreads();
    uint32_t rank[kRows];
    uint32_t dg[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        rank[r] = 0;
        dg[r] = 0;
        if ((uint32_t)r < rows) {      // uniform over the wave
            const uint32_t idx = w * cw + r * kWave + lane;
            const bool valid = idx < n;
            const uint32_t d = valid ? dig((K)(sk[idx] - kbase), shift) : 0u;
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
            dg[r] = d;
        }
    }
    __syncthreads();
    {
        const uint32_t d = threadIdx.x;
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < kW; ++ww) {
            const uint32_t t = whist[ww][d];
            whist[ww][d] = c;
            c += t;
        }
        uint32_t all;
        start[d] = block_exclusive_scan<uint32_t, kT>(c, scratch, &all);
        if (d == 0) start[256] = all;
        if (c) atomicMax(max_count, c);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        if ((uint32_t)r < rows) {
            const uint32_t idx = w * cw + r * kWave + lane;
            if (idx < n) {
                const uint32_t pos = start[dg[r]] + whist[w][dg[r]] + rank[r];
                dk[pos] = sk[idx];
                di[pos] = si ? si[idx] : (uint16_t)idx;
            }
        }
    }
    __syncthreads();
}

// Fast path, one workgroup per sub-bucket of at most kCap keys: keys stay in
// registers, are dropped into their group (next kGB bits) in LDS in any order,
// and each key's rank inside its group is counted by (key, input index), or
// by (key, place in the group) for keys without payload.
// Sub-buckets with a group larger than kGroupMax go to the LDS-LSD list,
// larger than kCap to the oversize list.
// Work of the small sort: entries [0, n_msd) are the sub-buckets of the MSD
// pass (entry = 256 * pass segment + digit), entries [n_msd, n_msd +
// n_direct) whole segments taken straight from their input.
template <typename K>
struct SmallJobs {
    uint32_t n_msd = 0;
    const uint32_t* msd_seg = nullptr;     // pass segment -> segment (nullptr: the same)
    const uint32_t* direct_seg = nullptr;
    const uint64_t* direct_src = nullptr;  // device addresses (nullptr: keys_in + position)
    const uint64_t* direct_vsrc = nullptr;
    const K* keys_in = nullptr;
    const uint64_t* vals_in = nullptr;
    K* stash = nullptr;                    // the MSD buffer: direct segments put on the slow list
    uint64_t* vstash = nullptr;
    const uint64_t* seg_off = nullptr;     // positions of every segment
    int key_bits = 64;
};

template <typename K, bool kPayload, int kCapT, int kGB>
__global__ __launch_bounds__(kT) void small_sort_kernel(const K* __restrict__ kin,
                                                        const uint64_t* __restrict__ vin,
                                                        K* __restrict__ kout,
                                                        uint64_t* __restrict__ vout,
                                                        const uint64_t* __restrict__ sb_start,
                                                        const uint32_t* __restrict__ sb_len,
                                                        int uniform_bits,
                                                        const uint8_t* __restrict__ seg_shift,
                                                        const uint64_t* __restrict__ seg_base,
                                                        OversizeList ov, SlowList sl,
                                                        SmallJobs<K> jobs, Fences fences) {
    constexpr int kRowsT = kCapT / kT;
    constexpr uint32_t kG = 1u << kGB;           // groups
    constexpr int kGR = (int)kG / kT;            // groups per thread in the scan
    static_assert(kGR >= 1 && kGR * kT == (int)kG, "group count");
    __shared__ K Bk[kCapT];
    __shared__ uint16_t Bi[kPayload ? kCapT : 1];   // input index of each placed key
    __shared__ uint32_t hist[kG];                 // group sizes
    __shared__ uint32_t cursor[kG];               // group starts, then ends after placement
    __shared__ uint32_t scratch[kW];
    __shared__ uint32_t max_count;

    uint64_t base;
    uint32_t n, seg;
    K kbase;
    int bits;
    const K* src;
    const uint64_t* vsrc;
    const bool direct = blockIdx.x >= jobs.n_msd;
    if (!direct) {
        base = sb_start[blockIdx.x];
        n = sb_len[blockIdx.x];
        const uint32_t li = blockIdx.x / 256;
        seg = jobs.msd_seg ? jobs.msd_seg[li] : li;
        kbase = seg_base ? (K)seg_base[seg] : (K)0;
        bits = seg_shift ? (int)seg_shift[seg] : uniform_bits;
        src = kin + base;
        vsrc = kPayload ? vin + base : nullptr;
    } else {
        const uint32_t dj = blockIdx.x - jobs.n_msd;
        seg = jobs.direct_seg[dj];
        base = jobs.seg_off[seg];
        n = (uint32_t)(jobs.seg_off[seg + 1] - base);
        kbase = (K)0;
        bits = jobs.key_bits;
        src = jobs.direct_src ? (const K*)(uintptr_t)jobs.direct_src[dj] : jobs.keys_in + base;
        vsrc = kPayload ? (jobs.direct_vsrc ? (const uint64_t*)(uintptr_t)jobs.direct_vsrc[dj]
                                            : jobs.vals_in + base)
                        : nullptr;
    }
    if (n == 0) return;
    if (n > (uint32_t)kCapT) {   // sub-buckets of the MSD pass only
        if (threadIdx.x == 0) {
            const uint32_t e = atomicAdd(ov.count, 1u);
            ov.beg[e] = base;
            ov.end[e] = base + n;
            ov.base[e] = (uint64_t)kbase;
            ov.seg[e] = seg;
        }
        return;
    }
    if (n == 1) {
        if (threadIdx.x == 0) {
            const K k = src[0];
            kout[base] = k;
            if constexpr (kPayload) vout[base] = vsrc[0];
            const FenceSink fs = fence_sink(fences, seg);
            if (fs.dst) put_fence(fs, base, (uint64_t)k);
        }
        return;
    }
    // the offsets key - kbase of this sub-bucket agree on every bit at or
    // above `bits`
    const int shift2 = bits >= kGB ? bits - kGB : 0;
    for (uint32_t i = threadIdx.x; i < kG; i += kT) hist[i] = 0;
    if (threadIdx.x == 0) max_count = 0;
    __syncthreads();
    K kr[kRowsT];
    uint32_t dr[kRowsT];
#pragma unroll
    for (int r = 0; r < kRowsT; ++r) {
        const uint32_t i = r * kT + threadIdx.x;
        kr[r] = 0;
        dr[r] = 0;
        if (i < n) kr[r] = src[i];
    }
#pragma unroll
    for (int r = 0; r < kRowsT; ++r) {
        const uint32_t i = r * kT + threadIdx.x;
        if (i < n) {
            dr[r] = (uint32_t)((K)(kr[r] - kbase) >> shift2) & (kG - 1);
            atomicAdd(&hist[dr[r]], 1u);
        }
    }
    __syncthreads();
    {
        // thread t scans the groups [t kGR, (t+1) kGR)
        uint32_t c[kGR], local = 0, mx = 0;
#pragma unroll
        for (int j = 0; j < kGR; ++j) {
            c[j] = hist[threadIdx.x * kGR + j];
            local += c[j];
            mx = max(mx, c[j]);
        }
        uint32_t all;
        uint32_t st = block_exclusive_scan<uint32_t, kT>(local, scratch, &all);
#pragma unroll
        for (int j = 0; j < kGR; ++j) {
            cursor[threadIdx.x * kGR + j] = st;
            st += c[j];
        }
        if (mx > kGroupMax) atomicMax(&max_count, mx);
    }
    __syncthreads();
    if (max_count > kGroupMax) {
        if (direct) {
            // the slow path reads the MSD buffer: move the segment there
#pragma unroll
            for (int r = 0; r < kRowsT; ++r) {
                const uint32_t i = r * kT + threadIdx.x;
                if (i < n) {
                    jobs.stash[base + i] = kr[r];
                    if constexpr (kPayload) jobs.vstash[base + i] = vsrc[i];
                }
            }
        }
        if (threadIdx.x == 0) {
            const uint32_t e = atomicAdd(sl.count, 1u);
            sl.beg[e] = base;
            sl.len[e] = n;
            sl.bits[e] = (uint8_t)bits;
            sl.base[e] = (uint64_t)kbase;
            sl.seg[e] = seg;
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < kRowsT; ++r) {
        const uint32_t i = r * kT + threadIdx.x;
        if (i < n) {
            const uint32_t pos = atomicAdd(&cursor[dr[r]], 1u);
            Bk[pos] = kr[r];
            if constexpr (kPayload) Bi[pos] = (uint16_t)i;
        }
    }
    __syncthreads();
    const FenceSink fs = fence_sink(fences, seg);
    for (uint32_t e = threadIdx.x; e < n; e += kT) {
        const K k = Bk[e];
        const uint32_t d = (uint32_t)((K)(k - kbase) >> shift2) & (kG - 1);
        const uint32_t g1 = cursor[d], g0 = g1 - hist[d];
        uint32_t rk = 0;
        if constexpr (kPayload) {
            // equal keys keep their input order
            const uint16_t ie = Bi[e];
            for (uint32_t j = g0; j < g1; ++j) {
                const K x = Bk[j];
                rk += (x < k || (x == k && Bi[j] < ie)) ? 1u : 0u;
            }
            const uint64_t o = base + g0 + rk;
            kout[o] = k;
            vout[o] = vsrc[ie];
            if (fs.dst) put_fence(fs, o, (uint64_t)k);
        } else {
            // keys only: equal keys are interchangeable, so the ones placed
            // before this one in the group go first
            for (uint32_t j = g0; j < e; ++j) rk += Bk[j] <= k ? 1u : 0u;
            for (uint32_t j = e + 1; j < g1; ++j) rk += Bk[j] < k ? 1u : 0u;
            const uint64_t o = base + g0 + rk;
            kout[o] = k;
            if (fs.dst) put_fence(fs, o, (uint64_t)k);
        }
    }
}

// Sub-buckets of at most kCap keys with a large group (duplicates or
// clustered keys): LSD counting passes in LDS over the digits below `bits`
// that vary, from the input order.
template <typename K, bool kPayload>
__global__ __launch_bounds__(kT) void lds_lsd_kernel(const K* __restrict__ kin,
                                                     const uint64_t* __restrict__ vin,
                                                     K* __restrict__ kout,
                                                     uint64_t* __restrict__ vout, SlowList sl,
                                                     Fences fences) {
    __shared__ K A[kCap];
    __shared__ K Bk[kCap];
    __shared__ uint16_t Ai[kCap];
    __shared__ uint16_t Bi[kCap];
    __shared__ uint32_t whist[kW][256];
    __shared__ uint32_t start[257];
    __shared__ uint32_t scratch[kW];
    __shared__ uint32_t max_count;
    __shared__ uint32_t diff_lo, diff_hi;

    const uint64_t base = sl.beg[blockIdx.x];
    const uint32_t n = sl.len[blockIdx.x];
    const int bits = sl.bits[blockIdx.x];
    const K kbase = (K)sl.base[blockIdx.x];
    if (threadIdx.x == 0) { diff_lo = 0; diff_hi = 0; }
    for (uint32_t i = threadIdx.x; i < n; i += kT) A[i] = kin[base + i];
    __syncthreads();
    {
        const uint64_t k0 = (uint64_t)(K)(A[0] - kbase);
        uint64_t acc = 0;
        for (uint32_t i = threadIdx.x; i < n; i += kT) acc |= (uint64_t)(K)(A[i] - kbase) ^ k0;
        if (acc) {
            atomicOr(&diff_lo, (uint32_t)acc);
            atomicOr(&diff_hi, (uint32_t)(acc >> 32));
        }
    }
    __syncthreads();
    const uint64_t diff = ((uint64_t)diff_hi << 32) | diff_lo;
    const K* sk = A;
    const uint16_t* si = nullptr;
    K* dk = Bk;
    uint16_t* di = Bi;
    for (int sh = 0; sh < bits; sh += 8) {
        if (((diff >> sh) & 0xFFu) == 0) continue;   // uniform digit: order unchanged
        lds_pass<K>(sk, si, dk, di, n, sh, kbase, whist, start, scratch, &max_count);
        // the pass output becomes the next input; the buffer pair (keys,
        // indices) it read from becomes the next output
        K* old = (K*)sk;
        sk = dk;
        si = di;
        dk = old;
        di = old == A ? Ai : Bi;
    }
    const uint32_t seg = sl.seg[blockIdx.x];
    const FenceSink fs = fence_sink(fences, seg);
    for (uint32_t i = threadIdx.x; i < n; i += kT) {
        kout[base + i] = sk[i];
        if constexpr (kPayload) vout[base + i] = vin[base + (si ? si[i] : i)];
        if (fs.dst) put_fence(fs, base + i, (uint64_t)sk[i]);
    }
}

// Fences of the oversize sub-buckets, read back from the sorted output.
template <typename K>
__global__ void ov_fence_kernel(const K* __restrict__ kout, OversizeList ov, Fences fences) {
    const uint32_t E = *ov.count;
    for (uint32_t e = blockIdx.x; e < E; e += gridDim.x) {
        const uint32_t seg = ov.seg[e];
        const uint64_t sb = fences.seg_off[seg];
        const uint64_t first = sb + ((ov.beg[e] - sb + kFenceStride - 1) / kFenceStride) * kFenceStride;
        for (uint64_t o = first + (uint64_t)threadIdx.x * kFenceStride; o < ov.end[e];
             o += (uint64_t)blockDim.x * kFenceStride)
            fences.key[fences.base[seg] + (o - sb) / kFenceStride] = (uint64_t)kout[o];
    }
}

// Workgroup per segment: every kFenceStride-th key of the sorted segment.
template <typename K>
__global__ void fence_fill_kernel(const K* __restrict__ keys, Fences fences) {
    const uint32_t seg = blockIdx.x;
    const uint64_t sb = fences.seg_off[seg];
    const uint64_t len = fences.seg_off[seg + 1] - sb;
    const uint64_t nf = (len + kFenceStride - 1) / kFenceStride;
    for (uint64_t f = threadIdx.x; f < nf; f += blockDim.x)
        fences.key[fences.base[seg] + f] = (uint64_t)keys[sb + f * kFenceStride];
}

// One workgroup: tile offsets of the oversize list, and the list sizes the
// host reads back in one copy.
__global__ __launch_bounds__(1024) void ov_tiles_kernel(OversizeList ov, SlowList sl) {
    __shared__ uint32_t scratch[1024 / kWave];
    const uint32_t E = *ov.count;
    uint32_t run = 0;
    for (uint32_t c = 0; c < E; c += 1024) {
        const uint32_t e = c + threadIdx.x;
        const uint32_t nt = e < E ? (uint32_t)((ov.end[e] - ov.beg[e] + kSortTile - 1) / kSortTile) : 0u;
        uint32_t tot;
        const uint32_t pre = block_exclusive_scan<uint32_t, 1024>(nt, scratch, &tot);
        if (e < E) ov.tile0[e] = run + pre;
        run += tot;
    }
    if (threadIdx.x == 0) {
        ov.tile0[E] = run;
        *ov.tiles = run;
        ov.summary[0] = E;
        ov.summary[1] = run;
        ov.summary[2] = *sl.count;
        ov.summary[3] = 0;
    }
}

__global__ void ov_fill_kernel(OversizeList ov) {
    const uint32_t E = *ov.count;
    for (uint32_t e = blockIdx.x; e < E; e += gridDim.x) {
        const uint32_t t0 = ov.tile0[e], t1 = ov.tile0[e + 1];
        for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) ov.tile_seg[t] = e;
    }
}

__global__ void ov_reset_kernel(OversizeList ov, SlowList sl) {
    *ov.count = 0;
    *ov.tiles = 0;
    *sl.count = 0;
}

}  // namespace

hipError_t hybrid_sort(const HybridSort& a, hipStream_t s, HybridHost& host) {
    const bool listed = a.msd_seg != nullptr;
    const uint32_t tps = listed ? 0u : (uint32_t)((a.max_seg_len + kSortTile - 1) / kSortTile);
    const uint32_t msd_segs = (listed || tps > 0) ? a.num_segs : 0u;
    const uint32_t msd_tiles = listed ? a.msd_tiles : msd_segs * tps;
    if (msd_segs == 0 && a.n_direct == 0) return hipSuccess;
    if (listed && (a.seg_shift || a.seg_base)) return hipErrorInvalidValue;
    const int kb = a.key_bytes * 8;
    const int bits = kb - 8;             // bits below the top digit
    Profiler dummy;
    Profiler& prof = a.prof ? *a.prof : dummy;
    const bool pay = a.vals_in != nullptr || a.has_payload;
    hipError_t e = hipSuccess;

    hipLaunchKernelGGL(ov_reset_kernel, dim3(1), dim3(1), 0, s, a.ov, a.sl);
    // 1. MSD pass of the large segments into the temporary buffer
    if (msd_segs > 0 && msd_tiles > 0) {
        RadixPass ps;
        ps.key_bytes = a.key_bytes;
        ps.keys_in = a.keys_in;
        ps.vals_in = a.vals_in;
        ps.keys_out = a.keys_tmp;
        ps.vals_out = a.vals_tmp;
        ps.map.beg = listed ? a.msd_beg : a.seg_off;
        ps.map.end = listed ? a.msd_end : a.seg_off + 1;
        ps.map.base = a.seg_base;
        ps.map.tile_seg = listed ? a.msd_tile_seg : nullptr;
        ps.map.tile0 = listed ? a.msd_tile0 : nullptr;
        ps.map.tps = tps;
        ps.map.src = a.msd_src;
        ps.map.vsrc = a.msd_vsrc;
        ps.num_segs = msd_segs;
        ps.num_tiles = msd_tiles;
        ps.shift = bits;
        ps.seg_shift = a.seg_shift;
        ps.counts = a.counts;
        ps.sb_start = a.sb_start;
        ps.sb_len = a.sb_len;
        ps.total_len = a.total_len;
        ps.prof = a.prof;
        // every sub-bucket is sorted completely afterwards; with keys only, equal
        // keys are interchangeable, so the order inside a run does not matter
        ps.any_order = !pay;
        ps.has_payload = pay;
        e = radix_pass(ps, s);
        if (e != hipSuccess) return e;
    }
    // 2. sub-buckets, and the segments small enough to take whole, in LDS
    const dim3 grid(msd_segs * 256u + a.n_direct);
    prof.begin(s);
    // sub-buckets of the p input segments split by their top byte average
    // N/(256 p) keys; bucket key ranges may use only half of the digit values
    const bool large = a.seg_base != nullptr;
#define HSS_SMALL(KT, PAY, CAP)                                                                  \
    do {                                                                                         \
        SmallJobs<KT> jobs;                                                                      \
        jobs.n_msd = msd_segs * 256u;                                                            \
        jobs.msd_seg = a.msd_seg;                                                                \
        jobs.direct_seg = a.direct_seg;                                                          \
        jobs.direct_src = a.direct_src;                                                          \
        jobs.direct_vsrc = a.direct_vsrc;                                                        \
        jobs.keys_in = (const KT*)a.keys_in;                                                     \
        jobs.vals_in = a.vals_in;                                                                \
        jobs.stash = (KT*)a.keys_tmp;                                                            \
        jobs.vstash = a.vals_tmp;                                                                \
        jobs.seg_off = a.seg_off;                                                                \
        jobs.key_bits = kb;                                                                      \
        hipLaunchKernelGGL((small_sort_kernel<KT, PAY, CAP, kGroupBits>), grid, dim3(kT), 0, s,  \
                           (const KT*)a.keys_tmp, PAY ? a.vals_tmp : nullptr, (KT*)a.keys_out,     \
                           PAY ? a.vals_out : nullptr, a.sb_start, a.sb_len, bits, a.seg_shift,    \
                           a.seg_base, a.ov, a.sl, jobs, a.fences);                                \
    } while (0)
    if (a.key_bytes == 4) {
        if (pay) { if (large) HSS_SMALL(uint32_t, true, kCapLarge); else HSS_SMALL(uint32_t, true, kCapSmall); }
        else { if (large) HSS_SMALL(uint32_t, false, kCapLarge); else HSS_SMALL(uint32_t, false, kCapSmall); }
    } else {
        if (pay) { if (large) HSS_SMALL(uint64_t, true, kCapLarge); else HSS_SMALL(uint64_t, true, kCapSmall); }
        else { if (large) HSS_SMALL(uint64_t, false, kCapLarge); else HSS_SMALL(uint64_t, false, kCapSmall); }
    }
#undef HSS_SMALL
    prof.end(kProfSmallSort, s, a.total_len * 2 * (a.key_bytes + (pay ? 8 : 0)));
    // 3. oversize sub-buckets: LSD passes in HBM over a compact list
    hipLaunchKernelGGL(ov_tiles_kernel, dim3(1), dim3(1024), 0, s, a.ov, a.sl);
    hipLaunchKernelGGL(ov_fill_kernel, dim3(1024), dim3(256), 0, s, a.ov);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(host.pinned, a.ov.summary, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const uint32_t E = host.pinned[0], T = host.pinned[1], SL = host.pinned[2];
    host.last_oversize = E;
    host.last_slow = SL;
    if (SL > 0) {
        const dim3 g(SL);
        if (a.key_bytes == 4) {
            if (pay) hipLaunchKernelGGL((lds_lsd_kernel<uint32_t, true>), g, dim3(kT), 0, s, (const uint32_t*)a.keys_tmp, a.vals_tmp, (uint32_t*)a.keys_out, a.vals_out, a.sl, a.fences);
            else hipLaunchKernelGGL((lds_lsd_kernel<uint32_t, false>), g, dim3(kT), 0, s, (const uint32_t*)a.keys_tmp, nullptr, (uint32_t*)a.keys_out, nullptr, a.sl, a.fences);
        } else {
            if (pay) hipLaunchKernelGGL((lds_lsd_kernel<uint64_t, true>), g, dim3(kT), 0, s, (const uint64_t*)a.keys_tmp, a.vals_tmp, (uint64_t*)a.keys_out, a.vals_out, a.sl, a.fences);
            else hipLaunchKernelGGL((lds_lsd_kernel<uint64_t, false>), g, dim3(kT), 0, s, (const uint64_t*)a.keys_tmp, nullptr, (uint64_t*)a.keys_out, nullptr, a.sl, a.fences);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (E == 0) return hipSuccess;
    const uint64_t words = (uint64_t)T * 256;
    if (words > host.fb_words) {
        if (host.fb_counts) (void)hipFree(host.fb_counts);
        host.fb_counts = nullptr;
        host.fb_words = 0;
        e = hipMalloc((void**)&host.fb_counts, words * 4);
        if (e != hipSuccess) return e;
        host.fb_words = words;
    }
    RadixPass fb;
    fb.key_bytes = a.key_bytes;
    fb.map.beg = a.ov.beg;
    fb.map.end = a.ov.end;
    fb.map.tile_seg = a.ov.tile_seg;
    fb.map.tile0 = a.ov.tile0;
    fb.map.base = a.ov.base;
    fb.num_segs = E;
    fb.num_tiles = T;
    fb.counts = host.fb_counts;
    fb.total_len = 0;
    fb.prof = a.prof;
    const int passes = (bits + 7) / 8;   // odd for 32- and 64-bit keys: ends in keys_out
    for (int i = 0; i < passes; ++i) {
        const bool from_tmp = (i % 2) == 0;
        fb.keys_in = from_tmp ? a.keys_tmp : a.keys_out;
        fb.vals_in = from_tmp ? a.vals_tmp : a.vals_out;
        fb.keys_out = from_tmp ? a.keys_out : a.keys_tmp;
        fb.vals_out = from_tmp ? a.vals_out : a.vals_tmp;
        if (!pay) { fb.vals_in = nullptr; fb.vals_out = nullptr; }
        fb.shift = 8 * i;
        e = radix_pass(fb, s);
        if (e != hipSuccess) return e;
    }
    if (a.fences.key) {
        if (a.key_bytes == 4)
            hipLaunchKernelGGL(ov_fence_kernel<uint32_t>, dim3(1024), dim3(256), 0, s, (const uint32_t*)a.keys_out, a.ov, a.fences);
        else
            hipLaunchKernelGGL(ov_fence_kernel<uint64_t>, dim3(1024), dim3(256), 0, s, (const uint64_t*)a.keys_out, a.ov, a.fences);
        e = hipGetLastError();
    }
    return e;
}

hipError_t write_fences(const void* keys, int key_bytes, uint32_t num_segs, const Fences& f,
                        hipStream_t s) {
    if (num_segs == 0 || !f.key) return hipSuccess;
    if (key_bytes == 4)
        hipLaunchKernelGGL(fence_fill_kernel<uint32_t>, dim3(num_segs), dim3(256), 0, s, (const uint32_t*)keys, f);
    else
        hipLaunchKernelGGL(fence_fill_kernel<uint64_t>, dim3(num_segs), dim3(256), 0, s, (const uint64_t*)keys, f);
    return hipGetLastError();
}

uint64_t oversize_capacity(uint32_t num_segs, uint64_t total_len) {
    const uint64_t by_count = (uint64_t)num_segs * 256;
    const uint64_t by_size = total_len / (kCapSmall + 1) + 1;
    return by_count < by_size ? by_count : by_size;
}

uint64_t slow_capacity(uint32_t num_segs, uint64_t total_len) {
    const uint64_t by_count = (uint64_t)num_segs * 256;
    const uint64_t by_size = total_len / (kGroupMax + 1) + 1;
    return by_count < by_size ? by_count : by_size;
}

uint64_t oversize_tile_capacity(uint32_t num_segs, uint64_t total_len) {
    return total_len / kSortTile + oversize_capacity(num_segs, total_len) + 1;
}

}  // namespace hss
