// Segmented stable sort by MSD splitting plus on-chip finishing.
//
//   1. one counting pass on the top 8 bits of the key (count / scan / scatter
//      of radix.hip) moves every segment into 256 sub-buckets, in the
//      temporary buffer; the scan records each sub-bucket's start and length.
//      The count pass also takes the AND and OR of the segment's keys: a
//      segment above the on-chip capacity whose top digit holds all its keys
//      skips the scatter and goes on with the bits that still vary (or, when
//      none does, is copied as it is)
//   2. one workgroup per sub-bucket of at most kCapT keys sorts it on chip by
//      the remaining bits and writes it to the output:
//        - the keys are dropped into groups by the next 9 bits in LDS, and
//          each key's place inside its group is counted directly (keys
//          smaller, or equal and earlier) unless that costs more than
//          kRankBudget comparisons per key;
//        - then the sub-bucket is listed for a second kernel that sorts
//          it by an on-chip sample sort: classes between and equal to the
//          distinct values of 64 sampled keys (a run of equal keys is placed
//          in one step), the keys of each unequal class ranked directly
//   3. sub-buckets above kCapT go through deeper levels of the same
//      count / scan / scatter pass on the 8 bits below their top.  An entry
//      (at the first level, a segment of at most 64 kCapT keys) whose digit
//      would leave most of its keys for another level takes splitters
//      instead: a key's "digit" is its class among up to 127 splitters drawn
//      from a sample of the entry (classes of keys equal to a splitter, and
//      between two), so a value repeated through the entry becomes one class
//      of equal keys, and the other classes hold about n / 128 keys each
//      whatever the bits look like.  Levels alternate between the temporary
//      buffer and the output; each level's sub-buckets are packed into
//      on-chip jobs of at most kCapT keys (the job's key range from its
//      first and last digit or class), and one still above kCapT takes
//      another level.
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
constexpr uint32_t kGroupMax = 32;           // groups up to this size never leave the fast path
// The fast path ranks each key against its group: sum over groups of size^2
// comparisons.  Above kRankBudget per key the slow path below is cheaper.
constexpr uint32_t kRankBudget = 64;
constexpr int kGroupBits = 9;                // bits of the second-level groups of the fast path

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

// Fast path, one workgroup per sub-bucket of at most kCapT keys: keys stay in
// registers, are dropped into their group (next kGB bits) in LDS in any order,
// and each key's rank inside its group is counted by (key, input index), or
// by (key, place in the group) for keys without payload.
// Sub-buckets whose large groups (above kGroupMax) would take more than
// kRankBudget comparisons per key go to the slow list, sub-buckets above
// kCapT to the oversize list.
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
    K* stash = nullptr;                    // the MSD buffer: slow-list entries are read from it
    uint64_t* vstash = nullptr;
    const uint64_t* seg_off = nullptr;     // positions of every segment
    int key_bits = 64;
    // packed jobs: job j is packed job j of `pj`, a run of sub-buckets of
    // entry li = pj.entry[j] of the level's list, whose keys were scattered
    // into the output (loc kLocTmp) or into the MSD buffer (otherwise); at
    // level 1 (lvl_seg null) of MSD pass segment li, in the MSD buffer
    PackedJobs pj;
    const uint32_t* lvl_seg = nullptr;
    const uint8_t* lvl_loc = nullptr;
    EqualList eq;                          // all-equal sub-buckets above the capacity
    // jobs of at most len_lo keys or of more than len_hi keys are another
    // launch's (the first level's sub-buckets split by size between the two
    // capacities)
    uint32_t len_lo = 0;
    uint32_t len_hi = ~0u;
};

// kStage: the payload is staged in LDS as well, so that a sub-bucket may be
// sorted in place (deeper levels, whose sub-buckets may already sit in the
// output).
template <typename K, bool kPayload, int kCapT, int kGB, bool kStage>
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
    static_assert(kPayload || !kStage, "staging is for the payload");
    constexpr int kRowsT = kCapT / kT;
    constexpr uint32_t kG = 1u << kGB;           // groups
    constexpr int kGR = (int)kG / kT;            // groups per thread in the scan
    static_assert(kGR >= 1 && kGR * kT == (int)kG, "group count");
    __shared__ K Bk[kCapT];
    __shared__ uint16_t Bi[kPayload ? kCapT : 1];   // input index of each placed key
    __shared__ uint64_t Bv[kStage ? kCapT : 1];     // payload of each placed key
    __shared__ uint32_t hist[kG];                 // group sizes
    __shared__ uint32_t cursor[kG];               // group starts, then ends after placement
    __shared__ uint32_t scratch[kW];
    __shared__ uint32_t max_count;
    __shared__ uint32_t rank_work;

    uint64_t base;
    uint32_t n, seg;
    K kbase;
    int bits;
    const K* src;
    const uint64_t* vsrc;
    bool in_out = false;   // the sub-bucket already sits in the output
    const bool direct = blockIdx.x >= jobs.n_msd;
    if (!direct) {
        if (jobs.pj.count) {
            // the grid is a bound on the packed jobs
            if (blockIdx.x >= min(*jobs.pj.count, jobs.pj.capacity)) return;
            base = jobs.pj.start[blockIdx.x];
            n = jobs.pj.len[blockIdx.x];
            const uint32_t li = jobs.pj.entry[blockIdx.x];
            if (jobs.lvl_seg) {
                seg = jobs.lvl_seg[li];
                in_out = jobs.lvl_loc[li] == kLocTmp;
            } else {   // level 1: entry li is MSD pass segment li, scattered into kin
                seg = jobs.msd_seg ? jobs.msd_seg[li] : li;
            }
            kbase = (K)jobs.pj.base[blockIdx.x];
            bits = jobs.pj.bits[blockIdx.x];
            src = (in_out ? (const K*)kout : kin) + base;
            vsrc = kPayload ? (in_out ? (const uint64_t*)vout : vin) + base : nullptr;
        } else {
            base = sb_start[blockIdx.x];
            n = sb_len[blockIdx.x];
            const uint32_t li = blockIdx.x / 256;
            seg = jobs.msd_seg ? jobs.msd_seg[li] : li;
            kbase = seg_base ? (K)seg_base[li] : (K)0;
            bits = seg_shift ? (int)seg_shift[li] : uniform_bits;
            src = kin + base;
            vsrc = kPayload ? vin + base : nullptr;
        }
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
    if (n <= jobs.len_lo || n > jobs.len_hi) return;   // uniform; also n == 0
    if (n > (uint32_t)kCapT) {   // sub-buckets of an MSD pass only
        if (threadIdx.x == 0) {
            if (bits == 0) {     // every key equal: nothing left to sort
                const uint32_t e = atomicAdd(jobs.eq.count, 1u);
                if (e >= jobs.eq.capacity) {
                    atomicOr(jobs.eq.err, 1u);
                    return;
                }
                jobs.eq.beg[e] = base;
                jobs.eq.end[e] = base + n;
                jobs.eq.seg[e] = seg;
                jobs.eq.loc[e] = in_out ? kLocOut : kLocTmp;
                jobs.eq.src[e] = (uint64_t)(uintptr_t)src;
                jobs.eq.vsrc[e] = (uint64_t)(uintptr_t)vsrc;
            } else {
                const uint32_t e = atomicAdd(ov.count, 1u);
                if (e >= ov.capacity) {
                    atomicOr(ov.err, 1u);
                    return;
                }
                ov.beg[e] = base;
                ov.end[e] = base + n;
                ov.base[e] = (uint64_t)kbase;
                ov.seg[e] = seg;
                ov.bits[e] = (uint8_t)bits;
                ov.loc[e] = in_out ? kLocOut : kLocTmp;
                ov.src[e] = (uint64_t)(uintptr_t)src;
                ov.vsrc[e] = (uint64_t)(uintptr_t)vsrc;
            }
        }
        return;
    }
    const FenceSink fs = fence_sink(fences, seg);
    if (n == 1 || bits == 0) {   // already in order: every key equal
        for (uint32_t i = threadIdx.x; i < n; i += kT) {
            const K k = as_global(src)[i];
            kout[base + i] = k;
            if constexpr (kPayload) vout[base + i] = as_global(vsrc)[i];
            if (fs.dst) put_fence(fs, base + i, (uint64_t)k);
        }
        return;
    }
    // the offsets key - kbase of this sub-bucket agree on every bit at or
    // above `bits`
    const int shift2 = bits >= kGB ? bits - kGB : 0;
    // a key's group; with 64-bit keys, no offset and the group bits in the
    // upper word (the first level of the local sort), one bit-field extract
    const bool hi_group = sizeof(K) == 8 && kbase == (K)0 && shift2 >= 32;
    auto group_of = [&](K k) -> uint32_t {
        if (hi_group) return __builtin_amdgcn_ubfe((uint32_t)((uint64_t)k >> 32), (uint32_t)(shift2 - 32), kGB);
        return (uint32_t)((K)(k - kbase) >> shift2) & (kG - 1);
    };
    for (uint32_t i = threadIdx.x; i < kG; i += kT) hist[i] = 0;
    if (threadIdx.x == 0) {
        max_count = 0;
        rank_work = 0;
    }
    __syncthreads();
    K kr[kRowsT];
    uint32_t dr[kRowsT];
    uint64_t vr[kStage ? kRowsT : 1];
    // rows wholly past the end are skipped by a branch uniform over the
    // workgroup; inside a row the lanes past the end hold kbase, whose group
    // is computed but never counted or placed
#pragma unroll
    for (int r = 0; r < kRowsT; ++r) {
        kr[r] = kbase;
        if (r * kT < (int)n) {
            const uint32_t i = r * kT + threadIdx.x;
            if (i < n) kr[r] = ld_stream(src + i);
            if constexpr (kStage) vr[r] = i < n ? ld_stream(vsrc + i) : 0;
        }
    }
#pragma unroll
    for (int r = 0; r < kRowsT; ++r) {
        dr[r] = 0;
        if (r * kT < (int)n) {
            dr[r] = group_of(kr[r]);
            if (r * kT + threadIdx.x < n) atomicAdd(&hist[dr[r]], 1u);
        }
    }
    __syncthreads();
    {
        // thread t scans the groups [t kGR, (t+1) kGR)
        uint32_t c[kGR], local = 0, mx = 0, sq = 0;
#pragma unroll
        for (int j = 0; j < kGR; ++j) {
            c[j] = hist[threadIdx.x * kGR + j];
            local += c[j];
            mx = max(mx, c[j]);
            sq += c[j] * c[j];
        }
        if (mx > kGroupMax) atomicAdd(&rank_work, sq);
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
    // bits <= kGB: a group holds one key value, so with keys alone the
    // placement below is already the sorted order
    const bool exact = !kPayload && bits <= kGB;
    // otherwise the groups above kGroupMax decide: their ranking work is
    // counted against the budget (small groups cost at most kGroupMax each)
    if (!exact && max_count > kGroupMax && rank_work > kRankBudget * n) {
        if (direct || in_out) {
            // the slow path reads the MSD buffer: move the keys there (its
            // copy of this range is no longer needed)
#pragma unroll
            for (int r = 0; r < kRowsT; ++r) {
                const uint32_t i = r * kT + threadIdx.x;
                if (i < n) {
                    jobs.stash[base + i] = kr[r];
                    if constexpr (kStage) jobs.vstash[base + i] = vr[r];
                    else if constexpr (kPayload) jobs.vstash[base + i] = as_global(vsrc)[i];
                }
            }
        }
        if (threadIdx.x == 0) {
            const uint32_t e = atomicAdd(sl.count, 1u);
            if (e >= sl.capacity) {
                atomicOr(sl.err, 1u);
                return;
            }
            sl.beg[e] = base;
            sl.len[e] = n;
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
            if constexpr (kStage) Bv[pos] = vr[r];
        }
    }
    __syncthreads();
    // outputs at offsets from the sub-bucket's start; a fence is due where the
    // offset from the segment start is a multiple of kFenceStride, which the
    // low 32 bits decide
    const uint64_t frel = fs.dst ? base - fs.org : 0;
    auto fence = [&](uint32_t o, K k) {
        if (fs.dst && (((uint32_t)frel + o) & (kFenceStride - 1)) == 0)
            fs.dst[(frel + o) / kFenceStride] = (uint64_t)k;
    };
    if (exact) {
        for (uint32_t e = threadIdx.x; e < n; e += kT) {
            const K k = Bk[e];
            st_stream(kout + base + e, k);
            fence(e, k);
        }
        return;
    }
    for (uint32_t e = threadIdx.x; e < n; e += kT) {
        const K k = Bk[e];
        const uint32_t d = group_of(k);
        const uint32_t g1 = cursor[d], g0 = g1 - hist[d];
        uint32_t rk = 0;
        if constexpr (kPayload) {
            // equal keys keep their input order
            const uint16_t ie = Bi[e];
            // the payload word is loaded while the rank is counted
            const uint64_t v = kStage ? Bv[e] : as_global(vsrc)[ie];
#pragma unroll 1
            for (uint32_t j = g0; j < g1; ++j) {
                const K x = Bk[j];
                rk += (uint32_t)((x < k) | ((x == k) & (Bi[j] < ie)));
            }
            const uint32_t o = g0 + rk;
            st_stream(kout + base + o, k);
            st_stream(vout + base + o, v);
            fence(o, k);
        } else {
            // keys only: equal keys are interchangeable, so the ones placed
            // before this one in the group go first; one pass over the group
            const K* const pe = Bk + g1;
            const K* const pk = Bk + e;
#pragma unroll 1
            for (const K* q = Bk + g0; q < pe; ++q) {
                const K x = *q;
                rk += (uint32_t)((x < k) | ((x == k) & (q < pk)));
            }
            const uint32_t o = g0 + rk;
            st_stream(kout + base + o, k);
            fence(o, k);
        }
    }
}

// Sub-buckets of at most kCap keys with large groups: runs of equal keys, or
// keys clustered in a few groups of their next bits.  An on-chip sample sort.
// Every key and payload is loaded once, into registers (wave w holds the keys
// [w cw, (w+1) cw) in rows of 64).  The distinct values S_0 < ... < S_{m-1}
// of 64 sampled keys split the keys into 2m + 1 classes in key order: class
// 2j + 1 holds the keys equal to S_j, class 2j those strictly between S_{j-1}
// and S_j.  A stable counting pass over the classes places every key: a class
// of equal keys is then in its final place (input order), and the keys of
// every other class are ranked against each other inside it (a class holds
// about n / 64 keys; one that the samples miss costs the square of its size,
// at most kCap^2 comparisons).  The places of those keys come back through
// LDS, and every key and payload is written from its register.
constexpr uint32_t kSlowSamples = kWave;

// Sample j: stratum j of 64 equal strata of the n keys, at an offset inside
// the stratum that varies with j (a permutation of the 64 residues), so that
// keys periodic in their position are sampled across their period.
__device__ __forceinline__ uint32_t sample_pos(uint32_t j, uint32_t n) {
    const uint32_t u = (j * 37u + 11u) & 63u;
    return (uint32_t)(((uint64_t)(kSlowSamples * j + u) * n) >> 12);
}

template <typename K>
__device__ __forceinline__ K shfl_key(K v, int src) {
    if constexpr (sizeof(K) == 8) return (K)shfl_u64((uint64_t)v, src);
    else return (K)__shfl((uint32_t)v, src);
}

template <typename K, bool kPayload, int kCap>
__global__ __launch_bounds__(kT) void sample_sort_kernel(const K* __restrict__ kin,
                                                     const uint64_t* __restrict__ vin,
                                                     K* __restrict__ kout,
                                                     uint64_t* __restrict__ vout, SlowList sl,
                                                     Fences fences) {
    constexpr int kRows = kCap / kT;   // rows of 64 keys per wave
    constexpr uint32_t kClasses = 2 * kSlowSamples + 1;
    static_assert(kSlowSamples == 64 && kClasses <= (uint32_t)kT, "one thread per class");
    __shared__ K Bk[kCap];            // the keys in input order, then the unequal classes
    __shared__ uint16_t Bi[kCap];     // input index of every key of an unequal class
    __shared__ uint16_t dest[kCap];   // input index -> place in the sub-bucket
    __shared__ uint8_t cpos[kCap];    // class of every place
    __shared__ uint32_t whist[kW][kClasses];
    __shared__ uint32_t start[kClasses + 1];
    __shared__ uint32_t scratch[kW];
    __shared__ K split[kSlowSamples];
    __shared__ uint32_t n_split;

    const uint64_t base = sl.beg[blockIdx.x];
    const uint32_t n = sl.len[blockIdx.x];
    const FenceSink fs = fence_sink(fences, sl.seg[blockIdx.x]);
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t cw = ((n + kW * kWave - 1) / (kW * kWave)) * kWave;
    const uint32_t rows = cw / kWave;
    auto index_of = [&](int r) { return w * cw + (uint32_t)r * kWave + lane; };
    K kr[kRows];
    uint64_t vr[kPayload ? kRows : 1];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        kr[r] = 0;
        if constexpr (kPayload) vr[r] = 0;
        if ((uint32_t)r < rows) {   // uniform over the workgroup
            const uint32_t i = index_of(r);
            if (i < n) {
                kr[r] = kin[base + i];
                if constexpr (kPayload) vr[r] = vin[base + i];
            }
        }
    }
    for (uint32_t i = threadIdx.x; i < kW * kClasses; i += kT) (&whist[0][0])[i] = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t i = index_of(r);
        if ((uint32_t)r < rows && i < n) Bk[i] = kr[r];
    }
    __syncthreads();
    if (w == 0) {
        // the samples sorted across the wave (bitonic network), then their
        // distinct values in order; the table is padded with the largest key,
        // which no key is below
        K v = Bk[sample_pos(lane, n)];
#pragma unroll
        for (uint32_t k = 2; k <= kSlowSamples; k <<= 1) {
#pragma unroll
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                const K x = shfl_key(v, (int)(lane ^ j));
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                v = keep_min ? (x < v ? x : v) : (x < v ? v : x);
            }
        }
        const K prev = shfl_key(v, (int)(lane == 0 ? 0 : lane - 1));
        const bool first = lane == 0 || prev != v;
        const uint64_t fm = __ballot(first);
        const uint32_t m = (uint32_t)__popcll(fm);
        if (first) split[__popcll(fm & lanes_below_mask())] = v;
        if (lane >= m) split[lane] = (K)~(K)0;
        if (lane == 0) n_split = m;
    }
    __syncthreads();
    const uint32_t m = n_split;
    // splitters below every key: binary lifting over the padded table, all
    // rows in step
    uint32_t lo[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) lo[r] = 0;
#pragma unroll
    for (uint32_t half = kSlowSamples / 2; half > 0; half >>= 1) {
#pragma unroll
        for (int r = 0; r < kRows; ++r)
            if ((uint32_t)r < rows && split[lo[r] + half - 1] < kr[r]) lo[r] += half;
    }
    // class of every key and its rank among the keys of its class in the
    // same wave, in input order (rows in order, lanes in order)
    uint32_t cl[kRows], pw[kRows];
    const uint64_t lanes_below = lanes_below_mask();
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        cl[r] = 0xFFu;
        pw[r] = 0;
        if ((uint32_t)r < rows) {   // uniform
            const bool valid = index_of(r) < n;
            const K k = kr[r];
            uint32_t s = lo[r];
            if (split[s] < k) ++s;   // s <= 63 before: all 64 below k
            const uint32_t c = 2 * s + ((s < m && split[s] == k) ? 1u : 0u);
            const uint64_t live = __ballot(valid);
            const uint64_t same = match_byte(c, live);
            const int leader = valid ? (int)(__ffsll((unsigned long long)same) - 1) : (int)lane;
            uint32_t old = 0;
            if (valid && (int)lane == leader) {
                old = whist[w][c];
                whist[w][c] = old + (uint32_t)__popcll(same);
            }
            old = __shfl(old, leader);
            if (valid) {
                cl[r] = c;
                pw[r] = old + (uint32_t)__popcll(same & lanes_below);
            }
        }
    }
    __syncthreads();
    {
        // class starts, and every wave's offset inside each class
        const uint32_t d = threadIdx.x;
        uint32_t c = 0;
        if (d < kClasses) {
#pragma unroll
            for (int ww = 0; ww < kW; ++ww) {
                const uint32_t t = whist[ww][d];
                whist[ww][d] = c;
                c += t;
            }
        }
        uint32_t all;
        const uint32_t st = block_exclusive_scan<uint32_t, kT>(c, scratch, &all);
        if (d < kClasses) start[d] = st;
        if (d == 0) start[kClasses] = all;
    }
    __syncthreads();
    // equal classes straight to their place; the others into LDS by class
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t c = cl[r];
        if (c == 0xFFu) continue;
        const uint32_t pos = start[c] + whist[w][c] + pw[r];
        if (c & 1u) {
            kout[base + pos] = kr[r];
            if constexpr (kPayload) vout[base + pos] = vr[r];
            if (fs.dst) put_fence(fs, base + pos, (uint64_t)kr[r]);
        } else {
            Bk[pos] = kr[r];
            Bi[pos] = (uint16_t)index_of(r);
        }
        cpos[pos] = (uint8_t)c;
    }
    __syncthreads();
    // every key of an unequal class: its rank inside the class (equal keys
    // of a class are in input order)
    for (uint32_t e = threadIdx.x; e < n; e += kT) {
        const uint32_t c = cpos[e];
        if (c & 1u) continue;
        const uint32_t g0 = start[c], g1 = start[c + 1];
        const K k = Bk[e];
        uint32_t rk = 0;
        for (uint32_t j = g0; j < g1; ++j) {
            const K x = Bk[j];
            rk += (uint32_t)((x < k) | ((x == k) & (j < e)));
        }
        dest[Bi[e]] = (uint16_t)(g0 + rk);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t c = cl[r];
        if (c == 0xFFu || (c & 1u)) continue;
        const uint32_t o = dest[index_of(r)];
        kout[base + o] = kr[r];
        if constexpr (kPayload) vout[base + o] = vr[r];
        if (fs.dst) put_fence(fs, base + o, (uint64_t)kr[r]);
    }
}

// Ranges whose keys are all equal: copied to the output unless already
// there, with their fences.  The range's key is read once; the payload is
// copied four words a thread at a time (all four loads in flight before the
// stores).  Workgroups stride over the entries.
template <typename K>
__global__ void equal_copy_kernel(K* __restrict__ kout, uint64_t* __restrict__ vout, EqualList eq,
                                  Fences fences) {
    constexpr uint32_t kG = 4;
    const uint32_t E = min(*eq.count, eq.capacity);
    for (uint32_t e = blockIdx.x; e < E; e += gridDim.x) {
        const uint64_t b = eq.beg[e], n = eq.end[e] - b;
        if (n == 0) continue;   // uniform over the workgroup
        const uint32_t seg = eq.seg[e];
        const FenceSink fs = fence_sink(fences, seg);
        const K k = *(const K*)(uintptr_t)eq.src[e];   // every key of the range
        const uint64_t* vsrc = (const uint64_t*)(uintptr_t)eq.vsrc[e];
        const bool copy = eq.loc[e] != kLocOut;
        if (!copy && !fs.dst) continue;   // in place, no fences: nothing to write
        for (uint64_t i0 = threadIdx.x; i0 < n; i0 += kG * blockDim.x) {
            uint64_t v[kG];
            if (copy && vout) {
#pragma unroll
                for (uint32_t q = 0; q < kG; ++q) {
                    const uint64_t i = i0 + (uint64_t)q * blockDim.x;
                    v[q] = i < n ? vsrc[i] : 0;
                }
            }
#pragma unroll
            for (uint32_t q = 0; q < kG; ++q) {
                const uint64_t i = i0 + (uint64_t)q * blockDim.x;
                if (i >= n) break;
                if (copy) {
                    kout[b + i] = k;
                    if (vout) vout[b + i] = v[q];
                }
                if (fs.dst) put_fence(fs, b + i, (uint64_t)k);
            }
        }
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

// One workgroup: tile offsets of an oversize list, and the list sizes the
// host reads back in one copy (entries, tiles, slow-list and equal-list
// entries).
__global__ __launch_bounds__(1024) void ov_tiles_kernel(OversizeList ov, SlowList sl, EqualList eq) {
    __shared__ uint32_t scratch[1024 / kWave];
    // a full list stops the sort: the overrun flag is read with the sizes
    const bool full = *ov.err != 0;
    const uint32_t E = full ? 0u : min(*ov.count, ov.capacity);
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
        ov.summary[2] = min(*sl.count, sl.capacity);
        ov.summary[3] = min(*eq.count, eq.capacity);
        ov.summary[4] = *ov.err;
        if (full) *ov.count = 0;
    }
}

__global__ void ov_fill_kernel(OversizeList ov) {
    const uint32_t E = min(*ov.count, ov.capacity);
    for (uint32_t e = blockIdx.x; e < E; e += gridDim.x) {
        const uint32_t t0 = ov.tile0[e], t1 = ov.tile0[e + 1];
        for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) ov.tile_seg[t] = e;
    }
}

// Empties a list; with the slow and equal lists given, also those and the
// overrun flag (start of a sort).
__global__ void ov_reset_kernel(OversizeList ov, SlowList sl, EqualList eq) {
    *ov.count = 0;
    *ov.tiles = 0;
    if (sl.count) *sl.count = 0;
    if (eq.count) {
        *eq.count = 0;
        *ov.err = 0;
    }
}

__global__ void count_reset_kernel(uint32_t* c) { *c = 0; }

// Level 1: the masks of every MSD segment start empty.
__global__ void mask_reset_kernel(LevelWork w, uint32_t n) {
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        w.and_mask[e] = ~0ull;
        w.or_mask[e] = 0;
        w.skip[e] = 0;
    }
}

// A deeper level over the entries of `ov`: each entry's digit is the 8 bits
// below its top (the lowest 8 when fewer remain), and its scatter goes to the
// other buffer (from the input, to the MSD buffer).
__global__ void level_prep_kernel(OversizeList ov, LevelWork w, uint64_t tmp, uint64_t out,
                                  uint64_t vtmp, uint64_t vout, int key_bytes) {
    const uint32_t E = min(*ov.count, ov.capacity);
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        const int bits = ov.bits[e];
        w.shift[e] = (uint8_t)(bits > 8 ? bits - 8 : 0);
        const bool to_out = ov.loc[e] == kLocTmp;
        w.dst[e] = (to_out ? out : tmp) + ov.beg[e] * (uint64_t)key_bytes;
        w.vdst[e] = vtmp ? (to_out ? vout : vtmp) + ov.beg[e] * 8 : 0;
        w.and_mask[e] = ~0ull;
        w.or_mask[e] = 0;
        w.skip[e] = 0;
    }
}

// The entries a level decides on: level 1 takes them from the MSD pass map
// (keys at the sort's input), deeper levels from their list.
struct DecideView {
    const uint64_t* beg = nullptr;
    const uint64_t* end = nullptr;
    const uint64_t* base = nullptr;    // null: 0
    const uint32_t* seg = nullptr;     // null: the entry index
    const uint8_t* loc = nullptr;      // null: kLocIn
    const uint64_t* src = nullptr;     // null: keys_in at beg
    const uint64_t* vsrc = nullptr;
    uint64_t keys_in = 0;
    uint64_t vals_in = 0;
    int key_bytes = 8;
    const uint32_t* count = nullptr;   // entries (null: n)
    uint32_t capacity = 0;             // of the list behind count
    uint32_t n = 0;
    uint32_t min_len = 0;              // entries of at most this many keys stay
    const uint8_t* shift = nullptr;    // digit of entry e at bits shift[e]..+7,
    int shift_all = 0;                 // or at shift_all when null
    // splitter levels: entry e's "digits" are its classes among the
    // n_splits[e] splitters of its table (kSplitSlots keys)
    const uint64_t* splits = nullptr;
    const uint32_t* n_splits = nullptr;
    // first level: entries of at most 64 look_cap keys take splitters when
    // most keys' digits would hold above look_cap keys (sub-buckets the level
    // would pass on); 0: when one digit holds a quarter of the keys
    uint32_t look_cap = 0;
    // first tile of entry e (its jobs are staged from slot 8 tile0[e] + e);
    // null: entries lie in order of position from 0 and the tile of beg[e]
    // plus e stands for it
    const uint32_t* tile0 = nullptr;
};

// First staging slot of entry e: room for 8 jobs per tile it spans and one
// more, below the first slot of any later entry.
__device__ inline uint64_t stage_slot(const DecideView& v, uint32_t e) {
    const uint64_t t = v.tile0 ? (uint64_t)v.tile0[e] : v.beg[e] / kSortTile + e;
    return 8 * t + e;
}

// Splitters of the entries of a level whose digit would leave most keys for
// another level, judged from 64 keys taken one per stratum of 64: at a deeper
// level (digit: the 8 bits below the entry's top, set by level_prep_kernel)
// when one digit value holds a quarter of them; at the first level (look_cap
// set) when half of them sit in digits estimated above look_cap keys.  Such
// an entry samples 128 keys (16 consecutive keys from a jittered
// place of each of 8 strata, one cache line a stratum), sorts them across the
// wave (bitonic network on lane shuffles, two keys a lane), and its distinct
// sample values, at most kSplitSlots - 1 of them, become its splitters S_0 <
// ... < S_{m-1}; the table is padded with all ones.  The level then places
// the entry's keys by their class among them instead of by the digit: a value
// with a key in the sample is one of the splitters, so its keys form a class
// of equal keys, sorted at once; the other classes hold about n / 128 keys
// each, however the key bits are spread.  Other entries keep their digit (no
// splitters).  A wave per entry; the waves stride over the entries.
template <typename K>
__global__ __launch_bounds__(256) void split_build_kernel(DecideView v, LevelWork w) {
    constexpr uint32_t kS = 2 * kWave;   // sample keys: element i is register i / 64 of lane i % 64
    constexpr uint32_t kRun = 16;        // consecutive keys per stratum
    static_assert(kS == kSplitSlots, "the distinct sample values fill at most the table");
    const uint32_t lane = lane_id();
    const uint64_t below = lanes_below_mask();
    const uint32_t E = v.count ? min(*v.count, v.capacity) : v.n;
    const uint32_t wpb = blockDim.x / kWave, waves = gridDim.x * wpb;
    for (uint32_t e = blockIdx.x * wpb + threadIdx.x / kWave; e < E; e += waves) {   // uniform over the wave
        const uint64_t n = v.end[e] - v.beg[e];
        if (n <= v.min_len || n < 2 * kSplitSlots || (v.look_cap && n > 64ull * v.look_cap)) {
            // sorted whole, too few keys to sample, or (first level) classes
            // of about n / 128 keys would not fit the small sort
            if (lane == 0) w.n_splits[e] = 0;
            continue;
        }
        const K* src = v.src ? (const K*)(uintptr_t)v.src[e]
                             : (const K*)(uintptr_t)(v.keys_in + v.beg[e] * (uint64_t)v.key_bytes);
        const K kb = v.base ? (K)v.base[e] : (K)0;
        const int shift = v.shift ? (int)v.shift[e] : v.shift_all;
        {
            const uint64_t u = (lane * 37u + 11u) & 63u;
            const K x = src[((64ull * lane + u) * n) / (64ull * kWave)];
            const uint32_t d = (uint32_t)((K)(x - kb) >> shift) & 0xFFu;
            const uint32_t c = (uint32_t)__popcll(match_byte(d, ~0ull));   // sampled keys in this digit
            bool split;
            if (v.look_cap) {
                // a sampled key's digit holds about c n / 64 keys: splitters
                // when half the sampled keys sit in digits above look_cap
                const bool big = (uint64_t)c * n > (uint64_t)kWave * v.look_cap;
                split = __popcll(__ballot(big)) >= kWave / 2;
            } else {
                split = __ballot(c >= kWave / 4) != 0;
            }
            if (!split) {   // uniform over the wave
                if (lane == 0) w.n_splits[e] = 0;
                continue;
            }
        }
        uint64_t v[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint64_t i = lane + kWave * q, st = i / kRun, u = (st * 37u + 11u) & 63u;
            const uint64_t at = min(((64ull * st + u) * n) / (64ull * (kS / kRun)), n - kRun);
            v[q] = (uint64_t)src[at + i % kRun];
        }
        for (uint32_t k = 2; k <= kS; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                if (j == kWave) {   // the pair (lane, lane + 64): this lane's two keys
                    const bool up = (lane & k) == 0;
                    const uint64_t lo = min(v[0], v[1]), hi = max(v[0], v[1]);
                    v[0] = up ? lo : hi;
                    v[1] = up ? hi : lo;
                } else {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const uint32_t i = lane + kWave * q;
                        const uint64_t y = shfl_u64(v[q], (int)(lane ^ j));
                        const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                        v[q] = keep_min ? min(v[q], y) : max(v[q], y);
                    }
                }
            }
        }
        // the distinct values in order: element i stays when i == 0 or it
        // differs from element i - 1 (the last element, rank 127, is left out)
        const uint64_t p0 = shfl_u64(v[0], (int)((lane + kWave - 1) % kWave));
        const uint64_t p1 = shfl_u64(v[1], (int)((lane + kWave - 1) % kWave));
        const uint64_t last0 = shfl_u64(v[0], kWave - 1);
        const bool keep0 = lane == 0 || v[0] != p0;
        const bool keep1 = lane + 1 < (uint32_t)kWave && v[1] != (lane == 0 ? last0 : p1);
        const uint64_t b0 = __ballot(keep0), b1 = __ballot(keep1);
        const uint32_t m0 = (uint32_t)__popcll(b0), m = m0 + (uint32_t)__popcll(b1);
        uint64_t* T = w.splits + (uint64_t)e * kSplitSlots;
        if (keep0) T[__popcll(b0 & below)] = v[0];
        if (keep1) T[m0 + __popcll(b1 & below)] = v[1];
        for (uint32_t c = m + lane; c < kSplitSlots; c += kWave) T[c] = ~0ull;
        if (lane == 0) {
            w.n_splits[e] = m;
            // a flag, not a count: one atomic per entry on one word would
            // take its turn with every other entry's
            if (*(volatile uint32_t*)w.split_entries == 0) *(volatile uint32_t*)w.split_entries = 1;
        }
    }
}


// Workgroup per entry, between scan and scatter.  When one digit holds all
// of an entry's keys the scatter would only copy them: the entry skips it,
// its sub-buckets are emptied, and it moves on with the bits that still vary
// (AND and OR of the count pass) -- to the equal list when none does, else to
// the next level's list with the highest varying bit as its new top.  The
// same holds when the top bits of the digit do not vary and even evenly
// filled sub-buckets would average more than twice the capacity: every one
// of them would take another level, so the entry takes that level whole, on
// the 8 bits below its highest varying bit (one scatter fewer).
// Deeper levels (pj given) also pack the entry's sub-buckets into small-sort
// jobs of at most `cap` keys, so that a level does not launch a workgroup per
// (mostly tiny) sub-bucket.
__global__ __launch_bounds__(256) void level_decide_kernel(DecideView v, LevelWork w,
                                                           const uint64_t* __restrict__ sb_start,
                                                           uint32_t* __restrict__ sb_len,
                                                           OversizeList next, EqualList eq,
                                                           PackedJobs pj, uint32_t cap) {
    __shared__ uint32_t nz;
    __shared__ uint32_t lens[256], starts[256];
    __shared__ uint32_t job_d0[256], job_d1[256], job_len[256];
    __shared__ uint32_t scan_tmp[256 / kWave];
    __shared__ int last_ne[256 / kWave];
    const uint32_t E = v.count ? min(*v.count, v.capacity) : v.n;
    const uint32_t e = blockIdx.x;
    if (e >= E) return;
    const uint64_t b = v.beg[e], n = v.end[e] - b;
    // entries of at most min_len keys are sorted as they are (packed into
    // jobs when pj is given)
    const bool small = n <= v.min_len;
    if (small && !pj.count) return;   // uniform over the workgroup
    if (threadIdx.x == 0) nz = 0;
    __syncthreads();
    const uint32_t len = sb_len[(uint64_t)e * 256 + threadIdx.x];
    lens[threadIdx.x] = len;
    if (len) atomicAdd(&nz, 1u);
    __syncthreads();
    bool narrow = false;
    const int sh = v.shift ? (int)v.shift[e] : v.shift_all;
    const bool by_splits = v.splits && v.n_splits[e] > 0;
    if (nz > 1 && !small && !by_splits) {   // uniform over the workgroup
        const uint64_t vary = w.and_mask[e] ^ w.or_mask[e];
        const int hb = 63 - __clzll((long long)vary);
        // 2^(hb - sh + 1) digit values can occur; each sub-bucket would
        // average n / 2^(hb - sh + 1) keys.  The next level's digit must lie
        // lower (its shift max(hb - 7, 0) is below sh only when sh > 0).
        narrow = vary != 0 && sh > 0 && hb >= sh && hb < sh + 7 && (n >> (hb - sh + 2)) > cap;
    }
    if (small || (nz != 1 && !narrow)) {
        if (!pj.count) return;
        // packing by windows of C = cap / 2 keys: a sub-bucket above C is a
        // job alone; the others form one job per run of sub-buckets whose
        // starts fall in the same window (less than 2 C = cap keys in all)
        const uint32_t C = cap / 2;
        const uint32_t d = threadIdx.x, lane = lane_id(), wv = d / kWave;
        uint32_t tot;
        const uint32_t st = block_exclusive_scan<uint32_t, 256>(len, scan_tmp, &tot);
        starts[d] = st;
        const bool ne = len != 0;
        const uint64_t mask = __ballot(ne);
        if (lane == 0) last_ne[wv] = mask ? (int)(wv * kWave + 63 - __clzll((long long)mask)) : -1;
        __syncthreads();
        // the previous non-empty sub-bucket: in this wave, else the last of
        // an earlier wave
        int pd = -1;
        const uint64_t below = mask & lanes_below_mask();
        if (below) {
            pd = (int)(wv * kWave + 63 - __clzll((long long)below));
        } else {
            for (int q = (int)wv - 1; q >= 0 && pd < 0; --q) pd = last_ne[q];
        }
        const bool big = len > C;
        const bool first = ne && (pd < 0 || big || lens[pd] > C || st / C != starts[pd] / C);
        // job index of every non-empty sub-bucket: inclusive count of firsts
        const uint32_t fi = block_exclusive_scan<uint32_t, 256>(first ? 1u : 0u, scan_tmp, &tot);
        const uint32_t jid = fi + (first ? 1u : 0u) - 1;   // valid where ne
        if (d < tot) {
            job_len[d] = 0;
            job_d0[d] = 0;   // last non-empty digit of the job
        }
        // an entry of t tiles gives at most 4 n / cap + 1 <= 8 t + 1 jobs
        // (cap >= 2048), the room its staging slots have
        const uint64_t q0 = stage_slot(v, e);
        const bool fits = tot <= 8 * ((n + kSortTile - 1) / kSortTile) + 1 && q0 + tot <= pj.s_capacity;
        if (d == 0) {
            pj.n_of[e] = fits ? tot : 0u;
            if (!fits) atomicOr(pj.err, 1u);
        }
        if (!fits) return;   // uniform over the workgroup
        __syncthreads();
        if (ne) {
            atomicAdd(&job_len[jid], len);
            atomicMax(&job_d0[jid], d);
            if (first) job_d1[jid] = d;   // first sub-bucket of the job
        }
        __syncthreads();
        const uint32_t nj = tot;
        const uint32_t shift = (uint32_t)sh;
        if (d < nj) {
            pj.s_start[q0 + d] = sb_start[(uint64_t)e * 256 + job_d1[d]];
            pj.s_len[q0 + d] = job_len[d];
            const uint64_t eb = v.base ? v.base[e] : 0;
            if (by_splits) {
                // the job's classes lie in [first, last]: its keys lie between
                // the least key the first class can hold and the largest the
                // last can (the entry's own ends from its AND and OR)
                const uint64_t* T = v.splits + (uint64_t)e * kSplitSlots;
                const uint32_t m = v.n_splits[e];
                const uint32_t c1 = job_d1[d], c0 = job_d0[d];
                const uint32_t j1 = c1 >> 1, j0 = c0 >> 1;
                // (the OR of the offsets may pass the largest key: the sum
                // is held to the key width)
                const uint64_t kmax = v.key_bytes == 4 ? 0xFFFFFFFFull : ~0ull;
                const uint64_t top = eb + w.or_mask[e];
                const uint64_t lo = (c1 & 1u) ? T[j1] : (j1 == 0 ? eb + w.and_mask[e] : T[j1 - 1] + 1);
                const uint64_t hi = (c0 & 1u) ? T[j0] : (j0 >= m ? (top < eb || top > kmax ? kmax : top) : T[j0] - 1);
                pj.s_base[q0 + d] = lo;
                pj.s_bits[q0 + d] = (uint8_t)(hi > lo ? 64 - __clzll((long long)(hi - lo)) : 0);
            } else {
                // the job's digits lie in [first, last]: taken from the first
                // digit on, key - base has digit (d - first) and the same bits
                // above the digit, so only the bits of last - first and those
                // below the digit vary (one sub-bucket: the bits below its digit)
                const uint32_t x = job_d0[d] - job_d1[d];
                pj.s_base[q0 + d] = eb + ((uint64_t)job_d1[d] << shift);
                pj.s_bits[q0 + d] = (uint8_t)(shift + (x ? 32 - __clz(x) : 0));
            }
        }
        return;
    }
    sb_len[(uint64_t)e * 256 + threadIdx.x] = 0;
    if (threadIdx.x != 0) return;
    if (pj.count) pj.n_of[e] = 0;
    w.skip[e] = 1;
    const uint32_t seg = v.seg ? v.seg[e] : e;
    const uint8_t loc = v.loc ? v.loc[e] : kLocIn;
    const uint64_t src = v.src ? v.src[e] : v.keys_in + b * (uint64_t)v.key_bytes;
    const uint64_t vsrc = v.vsrc ? v.vsrc[e] : (v.vals_in ? v.vals_in + b * 8 : 0);
    const uint64_t vary = w.and_mask[e] ^ w.or_mask[e];
    if (vary == 0) {
        const uint32_t q = atomicAdd(eq.count, 1u);
        if (q >= eq.capacity) {
            atomicOr(eq.err, 1u);
            return;
        }
        eq.beg[q] = b;
        eq.end[q] = b + n;
        eq.seg[q] = seg;
        eq.loc[q] = loc;
        eq.src[q] = src;
        eq.vsrc[q] = vsrc;
    } else {
        const uint32_t q = atomicAdd(next.count, 1u);
        if (q >= next.capacity) {
            atomicOr(next.err, 1u);
            return;
        }
        next.beg[q] = b;
        next.end[q] = b + n;
        next.base[q] = v.base ? v.base[e] : 0;
        next.seg[q] = seg;
        next.bits[q] = (uint8_t)(64 - __clzll((long long)vary));
        next.loc[q] = loc;
        next.src[q] = src;
        next.vsrc[q] = vsrc;
    }
}

// Packing of the staged jobs, in three launches: the job count of every
// chunk of kPackChunk entries (4 per thread); per chunk its offset (the
// counts of the chunks before it) and a scan of its entries, which turns
// n_of into each entry's first place in the list (n_of[E]: the list's size,
// stored by the first workgroup with the count); then the copy, a thread per
// job, each finding its entry among those places.
__global__ __launch_bounds__(256) void pack_count_kernel(PackedJobs pj, uint32_t E) {
    __shared__ uint32_t scratch[256 / kWave];
    const uint32_t i0 = blockIdx.x * kPackChunk + threadIdx.x * 4;
    uint32_t t = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
        if (i0 + k < E) t += pj.n_of[i0 + k];
    uint32_t tot;
    (void)block_exclusive_scan<uint32_t, 256>(t, scratch, &tot);
    if (threadIdx.x == 0) pj.chunk_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void pack_offsets_kernel(PackedJobs pj, uint32_t E) {
    __shared__ uint32_t scratch[256 / kWave];
    const uint32_t c = blockIdx.x;
    uint32_t before = 0, all = 0;
    for (uint32_t j = threadIdx.x; j < gridDim.x; j += 256) {
        const uint32_t x = pj.chunk_sum[j];
        if (j < c) before += x;
        all += x;
    }
    uint32_t off, tot;
    (void)block_exclusive_scan<uint32_t, 256>(before, scratch, &off);
    if (c == 0) {
        (void)block_exclusive_scan<uint32_t, 256>(all, scratch, &tot);
        if (threadIdx.x == 0) {
            *pj.count = tot;
            pj.n_of[E] = tot;
            if (tot > pj.capacity) atomicOr(pj.err, 1u);
        }
    }
    const uint32_t i0 = c * kPackChunk + threadIdx.x * 4;
    uint32_t cnt[4], t = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        cnt[k] = i0 + k < E ? pj.n_of[i0 + k] : 0u;
        t += cnt[k];
    }
    uint32_t q = off + block_exclusive_scan<uint32_t, 256>(t, scratch, &tot);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        if (i0 + k < E) pj.n_of[i0 + k] = q;
        q += cnt[k];
    }
}

__global__ __launch_bounds__(256) void pack_copy_kernel(PackedJobs pj, DecideView v, uint32_t E) {
    const uint32_t J = min(pj.n_of[E], pj.capacity);
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < J; q += gridDim.x * blockDim.x) {
        // the entry whose places hold q: the last e with n_of[e] <= q
        uint32_t lo = 0, hi = E - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (pj.n_of[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const uint64_t sl = stage_slot(v, lo) + (q - pj.n_of[lo]);
        pj.start[q] = pj.s_start[sl];
        pj.len[q] = pj.s_len[sl];
        pj.entry[q] = lo;
        pj.base[q] = pj.s_base[sl];
        pj.bits[q] = pj.s_bits[sl];
    }
}

template <typename K, bool kPay, int kCapT, bool kStage>
void launch_small(dim3 grid, hipStream_t s, const HybridSort& a, const uint64_t* sb_start,
                  const uint32_t* sb_len, int bits, const OversizeList& push, const SmallJobs<K>& jobs) {
    hipLaunchKernelGGL((small_sort_kernel<K, kPay, kCapT, kGroupBits, kStage>), grid, dim3(kT), 0, s,
                       (const K*)a.keys_tmp, kPay ? a.vals_tmp : nullptr, (K*)a.keys_out,
                       kPay ? a.vals_out : nullptr, sb_start, sb_len, bits, a.seg_shift, a.seg_base,
                       push, a.sl, jobs, a.fences);
}

// Level 1 (stage = false) reads sub-buckets from the MSD buffer; deeper
// levels may sort in place and stage the payload.
template <typename K>
void launch_small_any(bool pay, bool large, bool stage, dim3 grid, hipStream_t s,
                      const HybridSort& a, const uint64_t* sb_start, const uint32_t* sb_len,
                      int bits, const OversizeList& push, const SmallJobs<K>& jobs) {
    if (pay) {
        if (stage) {
            if (large) launch_small<K, true, kCapLarge, true>(grid, s, a, sb_start, sb_len, bits, push, jobs);
            else launch_small<K, true, kCapSmall, true>(grid, s, a, sb_start, sb_len, bits, push, jobs);
        } else {
            if (large) launch_small<K, true, kCapLarge, false>(grid, s, a, sb_start, sb_len, bits, push, jobs);
            else launch_small<K, true, kCapSmall, false>(grid, s, a, sb_start, sb_len, bits, push, jobs);
        }
    } else {
        if (large) launch_small<K, false, kCapLarge, false>(grid, s, a, sb_start, sb_len, bits, push, jobs);
        else launch_small<K, false, kCapSmall, false>(grid, s, a, sb_start, sb_len, bits, push, jobs);
    }
}

template <typename K, int kCapT>
void launch_sample_sort(bool pay, dim3 g, hipStream_t s, const HybridSort& a) {
    if (pay)
        hipLaunchKernelGGL((sample_sort_kernel<K, true, kCapT>), g, dim3(kT), 0, s, (const K*)a.keys_tmp,
                           a.vals_tmp, (K*)a.keys_out, a.vals_out, a.sl, a.fences);
    else
        hipLaunchKernelGGL((sample_sort_kernel<K, false, kCapT>), g, dim3(kT), 0, s, (const K*)a.keys_tmp,
                           nullptr, (K*)a.keys_out, nullptr, a.sl, a.fences);
}

template <typename K>
SmallJobs<K> level1_jobs(const HybridSort& a, uint32_t msd_segs, int kb) {
    SmallJobs<K> jobs;
    jobs.n_msd = msd_segs * 256u;
    jobs.msd_seg = a.msd_seg;
    jobs.direct_seg = a.direct_seg;
    jobs.direct_src = a.direct_src;
    jobs.direct_vsrc = a.direct_vsrc;
    jobs.keys_in = (const K*)a.keys_in;
    jobs.vals_in = a.vals_in;
    jobs.stash = (K*)a.keys_tmp;
    jobs.vstash = a.vals_tmp;
    jobs.seg_off = a.seg_off;
    jobs.key_bits = kb;
    jobs.eq = a.eq;
    return jobs;
}

template <typename K>
SmallJobs<K> level_jobs(const HybridSort& a, const OversizeList& cur, uint32_t grid) {
    SmallJobs<K> jobs;
    jobs.n_msd = grid;
    jobs.stash = (K*)a.keys_tmp;
    jobs.vstash = a.vals_tmp;
    jobs.seg_off = a.seg_off;
    jobs.pj = a.pj;
    jobs.lvl_seg = cur.seg;
    jobs.lvl_loc = cur.loc;
    jobs.eq = a.eq;
    return jobs;
}

__global__ void fill_zero_kernel(uint32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t read_summary(const OversizeList& ov, const SlowList& sl, const EqualList& eq,
                        HybridHost& host, hipStream_t s) {
    hipLaunchKernelGGL(ov_tiles_kernel, dim3(1), dim3(1024), 0, s, ov, sl, eq);
    hipLaunchKernelGGL(ov_fill_kernel, dim3(1024), dim3(256), 0, s, ov);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host.pinned, ov.summary, 5 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && host.pinned[4]) e = hipErrorOutOfMemory;   // a list overran
    return e;
}

// Splitters for the entries of a level whose digit would leave most of their
// keys for another level; the level takes the splitter kernels only when one
// entry has them (a flag read back).
hipError_t launch_splits(const HybridSort& a, const DecideView& v, uint32_t E, HybridHost& host, hipStream_t s) {
    const dim3 grid(min((E + 3) / 4, 16384u));
    hipLaunchKernelGGL(count_reset_kernel, dim3(1), dim3(1), 0, s, a.lw.split_entries);
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(split_build_kernel<uint32_t>, grid, dim3(256), 0, s, v, a.lw);
    else
        hipLaunchKernelGGL(split_build_kernel<uint64_t>, grid, dim3(256), 0, s, v, a.lw);
    return hipMemcpyAsync(host.pinned + 5, a.lw.split_entries, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
}

hipError_t build_splits(const HybridSort& a, const DecideView& v, uint32_t E, HybridHost& host, hipStream_t s,
                        bool* by_splits) {
    hipError_t e = launch_splits(a, v, E, host, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    *by_splits = e == hipSuccess && host.pinned[5] > 0;
    return e;
}

// The staged jobs of a level's E entries into the packed list.
void pack_jobs(const PackedJobs& pj, const DecideView& v, uint32_t E, hipStream_t s) {
    const uint32_t g = (E + kPackChunk - 1) / kPackChunk;
    hipLaunchKernelGGL(pack_count_kernel, dim3(g), dim3(256), 0, s, pj, E);
    hipLaunchKernelGGL(pack_offsets_kernel, dim3(g), dim3(256), 0, s, pj, E);
    hipLaunchKernelGGL(pack_copy_kernel, dim3(1024), dim3(256), 0, s, pj, v, E);
}

template <typename T>
hipError_t grow(MemSource* mem, T** p, uint64_t* cap, uint64_t need) {
    if (need <= *cap) return hipSuccess;
    if (*p) dev_release(mem, *p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = dev_alloc(mem, (void**)p, need * sizeof(T));
    if (e == hipSuccess) *cap = need;
    return e;
}

}  // namespace

hipError_t hybrid_sort(const HybridSort& a, hipStream_t s, HybridHost& host) {
    const bool listed = a.msd_seg != nullptr;
    const uint32_t tps = listed ? 0u : (uint32_t)((a.max_seg_len + kSortTile - 1) / kSortTile);
    const uint32_t msd_segs = (listed || tps > 0) ? a.num_segs : 0u;
    const uint32_t msd_tiles = listed ? a.msd_tiles : msd_segs * tps;
    if (msd_segs == 0 && a.n_direct == 0) return hipSuccess;
    const int kb = a.key_bytes * 8;
    const int bits = kb - 8;             // bits below the top digit
    Profiler dummy;
    Profiler& prof = a.prof ? *a.prof : dummy;
    const bool pay = a.vals_in != nullptr || a.has_payload;
    // sub-buckets of the p input segments split by their top byte average
    // N/(256 p) keys; bucket key ranges may use only half of the digit values
    const bool large = a.seg_base != nullptr || a.cap_large;
    const uint32_t cap = large ? kCapLarge : kCapSmall;
    hipError_t e = hipSuccess;

    hipLaunchKernelGGL(ov_reset_kernel, dim3(1), dim3(1), 0, s, a.ov, a.sl, a.eq);
    // Sub-buckets averaging under a quarter of the capacity (many segments
    // of few keys) are packed into jobs of up to `cap` keys, as at the
    // deeper levels, so that the small sort does not spend a workgroup on
    // every few hundred keys.  An entry of n keys gives at most 4 n / cap + 1
    // jobs.
    const uint64_t msd_keys = listed ? (uint64_t)msd_tiles * kSortTile : a.total_len;
    const uint64_t job_bound1 = 4 * msd_keys / cap + msd_segs;
    const bool can_pack1 = msd_segs > 0 && msd_tiles > 0 && a.pj.count && job_bound1 <= a.pj.capacity;
    bool pack1 = can_pack1 && msd_keys < (uint64_t)msd_segs * 256 * (cap / 4);
    // 1. MSD pass of the large segments into the temporary buffer.  A segment
    //    above the small-sort capacity whose top digit holds all its keys
    //    skips the scatter and goes on to the deeper levels.
    if (msd_segs > 0 && msd_tiles > 0) {
        DecideView v;
        v.beg = listed ? a.msd_beg : a.seg_off;
        v.end = listed ? a.msd_end : a.seg_off + 1;
        v.base = a.seg_base;
        v.seg = a.msd_seg;
        v.src = a.msd_src;
        v.vsrc = a.msd_vsrc;
        v.keys_in = (uint64_t)(uintptr_t)a.keys_in;
        v.vals_in = (uint64_t)(uintptr_t)a.vals_in;
        v.key_bytes = a.key_bytes;
        v.n = msd_segs;
        v.min_len = cap;
        v.shift = a.seg_shift;
        v.shift_all = bits;
        v.tile0 = listed ? a.msd_tile0 : nullptr;
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
        ps.map.skip = a.lw.skip;
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
        ps.and_mask = a.lw.and_mask;
        ps.or_mask = a.lw.or_mask;
        ps.counted = a.counted;
        if (!a.counted)
            hipLaunchKernelGGL(mask_reset_kernel, dim3(min((msd_segs + 255) / 256, 1024u)), dim3(256), 0, s,
                               a.lw, msd_segs);
        // A segment of few distinct digits, whose sub-buckets would mostly
        // pass to the next level, takes splitters here (its sub-buckets then
        // go through packed jobs, which carry their key ranges); not when the
        // digits were counted already by the kernel that wrote the keys.
        // Unless the plan's last call took them, the count by digits is
        // queued behind the flag's copy and the host waits for the copy
        // alone; with splitters the count is taken again by class.
        bool by_splits = false, counted_digits = false;
        if (can_pack1 && !a.counted && (a.min_seg_len == 0 || a.min_seg_len <= 64ull * cap)) {
            v.look_cap = cap;
            e = launch_splits(a, v, msd_segs, host, s);
            if (e == hipSuccess && host.flag_ev && !host.split1_last) {
                e = hipEventRecord(host.flag_ev, s);
                if (e == hipSuccess) e = radix_count_scan(ps, s);
                if (e == hipSuccess) e = hipEventSynchronize(host.flag_ev);
                counted_digits = true;
            } else if (e == hipSuccess) {
                e = hipStreamSynchronize(s);
            }
            if (e != hipSuccess) return e;
            by_splits = host.pinned[5] > 0;
            host.split1_last = by_splits;
            pack1 = pack1 || by_splits;
        }
        v.look_cap = 0;
        v.splits = by_splits ? a.lw.splits : nullptr;
        v.n_splits = by_splits ? a.lw.n_splits : nullptr;
        ps.map.splits = v.splits;
        ps.map.n_splits = v.n_splits;
        if (!counted_digits || by_splits) {
            e = radix_count_scan(ps, s);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(level_decide_kernel, dim3(msd_segs), dim3(256), 0, s, v, a.lw, a.sb_start,
                           a.sb_len, a.ov, a.eq, pack1 ? a.pj : PackedJobs{}, cap);
        if (pack1) pack_jobs(a.pj, v, msd_segs, s);
        e = radix_scatter(ps, s);
        if (e != hipSuccess) return e;
    }
    // 2. sub-buckets (or their packed jobs), and the segments small enough to
    //    take whole, in LDS
    {
        const uint32_t n_first = pack1 ? (uint32_t)job_bound1 : msd_segs * 256u;
        const dim3 grid(n_first + a.n_direct);
        prof.begin(s);
        auto run = [&](auto key) {
            using K = decltype(key);
            SmallJobs<K> jobs = level1_jobs<K>(a, msd_segs, kb);
            if (pack1) {
                jobs.n_msd = n_first;
                jobs.pj = a.pj;
            }
            if (large && !pack1) {
                // sub-buckets within the small capacity take its kernel (fewer
                // keys per group to rank), the larger ones the large kernel
                SmallJobs<K> fit = jobs;
                fit.len_hi = kCapSmall;
                launch_small_any<K>(pay, false, false, grid, s, a, a.sb_start, a.sb_len, bits, a.ov, fit);
                jobs.len_lo = kCapSmall;
            }
            launch_small_any<K>(pay, large, false, grid, s, a, a.sb_start, a.sb_len, bits, a.ov, jobs);
        };
        if (a.key_bytes == 4) run(uint32_t{});
        else run(uint64_t{});
        prof.end(kProfSmallSort, s, a.total_len * 2 * (a.key_bytes + (pay ? 8 : 0)));
    }
    e = read_summary(a.ov, a.sl, a.eq, host, s);
    if (e != hipSuccess) return e;
    uint32_t E = host.pinned[0], T = host.pinned[1];
    host.last_oversize = E;
    host.last_levels = 0;
    // 3. deeper levels: every entry above the capacity takes an MSD pass on
    //    the 8 bits below its top, alternating between the MSD buffer and the
    //    output; each level lowers the top of every entry it keeps, so at
    //    most kb levels follow
    OversizeList cur = a.ov, nxt = a.ov2;
    while (E > 0) {
        if (++host.last_levels > (uint32_t)kb) return hipErrorUnknown;
        e = grow(host.mem, &host.fb_counts, &host.fb_words, (uint64_t)T * 256);
        if (e == hipSuccess) {
            uint64_t c0 = host.fb_sb;
            e = grow(host.mem, &host.fb_sb_start, &c0, (uint64_t)E * 256 + 1);
            if (e == hipSuccess) e = grow(host.mem, &host.fb_sb_len, &host.fb_sb, (uint64_t)E * 256 + 1);
        }
        if (e != hipSuccess) return e;
        const uint64_t kt = (uint64_t)(uintptr_t)a.keys_tmp, ko = (uint64_t)(uintptr_t)a.keys_out;
        const uint64_t vt = pay ? (uint64_t)(uintptr_t)a.vals_tmp : 0, vo = pay ? (uint64_t)(uintptr_t)a.vals_out : 0;
        hipLaunchKernelGGL(level_prep_kernel, dim3(min((E + 255) / 256, 1024u)), dim3(256), 0, s, cur, a.lw,
                           kt, ko, vt, vo, a.key_bytes);
        DecideView v;
        v.beg = cur.beg;
        v.end = cur.end;
        v.base = cur.base;
        v.seg = cur.seg;
        v.loc = cur.loc;
        v.src = cur.src;
        v.vsrc = cur.vsrc;
        v.key_bytes = a.key_bytes;
        v.count = cur.count;
        v.capacity = cur.capacity;
        v.shift = a.lw.shift;
        v.tile0 = cur.tile0;
        bool by_splits = false;
        e = build_splits(a, v, E, host, s, &by_splits);
        if (e != hipSuccess) return e;
        RadixPass ps;
        ps.key_bytes = a.key_bytes;
        ps.keys_in = a.keys_tmp;        // unused: every entry has its source
        ps.vals_in = pay ? a.vals_tmp : nullptr;
        ps.keys_out = a.keys_out;       // unused: every entry has its destination
        ps.vals_out = pay ? a.vals_out : nullptr;
        ps.map.beg = cur.beg;
        ps.map.end = cur.end;
        ps.map.base = cur.base;
        ps.map.tile_seg = cur.tile_seg;
        ps.map.tile0 = cur.tile0;
        ps.map.src = cur.src;
        ps.map.vsrc = pay ? cur.vsrc : nullptr;
        ps.map.dst = a.lw.dst;
        ps.map.vdst = pay ? a.lw.vdst : nullptr;
        ps.map.skip = a.lw.skip;
        ps.map.splits = by_splits ? a.lw.splits : nullptr;
        ps.map.n_splits = by_splits ? a.lw.n_splits : nullptr;
        ps.num_segs = E;
        ps.num_tiles = T;
        ps.seg_shift = a.lw.shift;
        ps.counts = host.fb_counts;
        ps.sb_start = host.fb_sb_start;
        ps.sb_len = host.fb_sb_len;
        ps.total_len = (uint64_t)T * kSortTile;   // bound for the byte counts
        ps.prof = a.prof;
        ps.any_order = !pay;
        ps.has_payload = pay;
        ps.and_mask = a.lw.and_mask;
        ps.or_mask = a.lw.or_mask;
        e = radix_count_scan(ps, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(ov_reset_kernel, dim3(1), dim3(1), 0, s, nxt, SlowList{}, EqualList{});
        v.splits = by_splits ? a.lw.splits : nullptr;
        v.n_splits = by_splits ? a.lw.n_splits : nullptr;
        hipLaunchKernelGGL(level_decide_kernel, dim3(E), dim3(256), 0, s, v, a.lw, host.fb_sb_start,
                           host.fb_sb_len, nxt, a.eq, a.pj, cap);
        pack_jobs(a.pj, v, E, s);
        e = radix_scatter(ps, s);
        if (e != hipSuccess) return e;
        // packed jobs: an entry of n keys gives at most n / (cap/2) jobs of
        // one large sub-bucket and n / (cap/2) + 1 windows
        const uint64_t job_bound = 4 * ((uint64_t)T * kSortTile) / cap + E;
        const dim3 grid((uint32_t)std::min<uint64_t>(job_bound, a.pj.capacity));
        prof.begin(s);
        if (a.key_bytes == 4)
            launch_small_any<uint32_t>(pay, large, pay, grid, s, a, host.fb_sb_start, host.fb_sb_len, 0, nxt,
                                       level_jobs<uint32_t>(a, cur, grid.x));
        else
            launch_small_any<uint64_t>(pay, large, pay, grid, s, a, host.fb_sb_start, host.fb_sb_len, 0, nxt,
                                       level_jobs<uint64_t>(a, cur, grid.x));
        prof.end(kProfSmallSort, s, ps.total_len * 2 * (a.key_bytes + (pay ? 8 : 0)));
        e = read_summary(nxt, a.sl, a.eq, host, s);
        if (e != hipSuccess) return e;
        E = host.pinned[0];
        T = host.pinned[1];
        const OversizeList t = cur;
        cur = nxt;
        nxt = t;
    }
    const uint32_t SL = host.pinned[2], EQ = host.pinned[3];
    host.last_slow = SL;
    // 4. sub-buckets with a large group: the slow path (from the MSD buffer)
    if (SL > 0) {
        const dim3 g(SL);
        if (a.key_bytes == 4) {
            if (large) launch_sample_sort<uint32_t, kCapLarge>(pay, g, s, a);
            else launch_sample_sort<uint32_t, kCapSmall>(pay, g, s, a);
        } else {
            if (large) launch_sample_sort<uint64_t, kCapLarge>(pay, g, s, a);
            else launch_sample_sort<uint64_t, kCapSmall>(pay, g, s, a);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // 5. ranges of equal keys: into the output, with their fences
    if (EQ > 0) {
        const dim3 g(min(EQ, 4096u));
        if (a.key_bytes == 4)
            hipLaunchKernelGGL(equal_copy_kernel<uint32_t>, g, dim3(256), 0, s, (uint32_t*)a.keys_out, pay ? a.vals_out : nullptr, a.eq, a.fences);
        else
            hipLaunchKernelGGL(equal_copy_kernel<uint64_t>, g, dim3(256), 0, s, (uint64_t*)a.keys_out, pay ? a.vals_out : nullptr, a.eq, a.fences);
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

// Entries of the oversize and equal lists are disjoint ranges of more than
// kCapSmall keys; slow-list entries disjoint ranges of more than kGroupMax.
hipError_t launch_sort_count_reset(uint32_t* counts, uint64_t words, LevelWork w, uint32_t n, hipStream_t s) {
    if (words) {
        const uint32_t grid = (uint32_t)std::min<uint64_t>((words + 255) / 256, 4096);
        hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, s, counts, words);
    }
    if (n) hipLaunchKernelGGL(mask_reset_kernel, dim3(std::min((n + 255) / 256, 1024u)), dim3(256), 0, s, w, n);
    return hipGetLastError();
}

uint64_t oversize_capacity(uint64_t total_len) { return total_len / (kCapSmall + 1) + 1; }

uint64_t slow_capacity(uint64_t total_len) { return total_len / (kGroupMax + 1) + 1; }

uint64_t oversize_tile_capacity(uint64_t total_len) {
    return total_len / kSortTile + oversize_capacity(total_len) + 1;
}

// Per-entry arrays serve level 1 (every MSD segment) and the deeper levels.
// Packed jobs: per entry at most 4 n / kCapSmall + 1, and at most
// oversize_capacity() entries.
uint64_t packed_capacity(uint64_t total_len) {
    return 4 * total_len / kCapSmall + oversize_capacity(total_len) + 1;
}

uint64_t level_capacity(uint32_t num_segs, uint64_t total_len) {
    const uint64_t o = oversize_capacity(total_len);
    return num_segs > o ? num_segs : o;
}

// Staging slots of the packed jobs: 8 per tile and one per entry, for the
// tiles of a level (at most total_len / kSortTile plus one per entry) or the
// tile of each entry's first position plus one per entry before it (level 1
// in fixed mode).
uint64_t stage_capacity(uint32_t num_segs, uint64_t total_len) {
    const uint64_t l = level_capacity(num_segs, total_len);
    return 8 * (total_len / kSortTile + l + 1) + l + 1;
}

}  // namespace hss
