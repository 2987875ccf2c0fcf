// Host-side interfaces between the executor (hss.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace hss {

constexpr uint64_t kNone = ~0ull;

// ------------------------------------------------------------ profiling ----
// Kernel families timed with HIP events on the launching stream when a plan
// has profiling switched on.  `bytes` accumulates the algorithmic bytes the
// launches move (reads + writes of keys, payload and tables).
enum ProfSlot : int {
    kProfRadixCount = 0,
    kProfRadixScan,
    kProfRadixScatter,
    kProfRounds,
    kProfExchangeOffsets,
    kProfExchangeCopy,
    kProfSmallSort,
    kProfSlots
};

struct Profiler {
    bool on = false;
    struct Pending {
        int slot;
        hipEvent_t a, b;
        uint64_t bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    double ms[kProfSlots] = {};
    uint64_t launches[kProfSlots] = {};
    uint64_t bytes[kProfSlots] = {};
    hipEvent_t open_a = nullptr;

    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!spare.empty()) {
            e = spare.back();
            spare.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    void begin(hipStream_t s) {
        if (!on) return;
        open_a = take();
        if (open_a) (void)hipEventRecord(open_a, s);
    }
    void end(int slot, hipStream_t s, uint64_t nbytes) {
        if (!on || !open_a) return;
        hipEvent_t b = take();
        if (!b) return;
        (void)hipEventRecord(b, s);
        pending.push_back({slot, open_a, b, nbytes});
        open_a = nullptr;
    }
    // Waits for the recorded events and folds them into the totals.
    void collect() {
        for (const Pending& q : pending) {
            float t = 0;
            if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&t, q.a, q.b) == hipSuccess) {
                ms[q.slot] += t;
                launches[q.slot] += 1;
                bytes[q.slot] += q.bytes;
            }
            spare.push_back(q.a);
            spare.push_back(q.b);
        }
        pending.clear();
    }
    void reset() {
        collect();
        for (int i = 0; i < kProfSlots; ++i) { ms[i] = 0; launches[i] = 0; bytes[i] = 0; }
    }
    ~Profiler() {
        for (const Pending& q : pending) { (void)hipEventDestroy(q.a); (void)hipEventDestroy(q.b); }
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    }
};

// ----------------------------------------------------------- radix sort ----
// Stable sort of every segment [seg_off[s], seg_off[s+1]) of a key array by
// bits [begin_bit, end_bit) of the key, moving an optional 64-bit payload.
// The first pass reads keys_in; the last pass writes keys_out; passes in
// between alternate between keys_tmp and keys_out.  keys_in must differ
// from keys_tmp and keys_out (it may be read-only memory).
struct SegSort {
    int key_bytes = 8;                 // 4 or 8
    const void* keys_in = nullptr;
    const uint64_t* vals_in = nullptr; // nullptr: keys only
    void* keys_out = nullptr;
    uint64_t* vals_out = nullptr;
    void* keys_tmp = nullptr;
    uint64_t* vals_tmp = nullptr;
    const uint64_t* seg_off = nullptr; // device, S+1 entries
    uint32_t num_segs = 0;
    uint64_t max_seg_len = 0;          // upper bound of every segment length
    uint64_t total_len = 0;            // sum of the segment lengths (for byte counts)
    uint32_t* counts = nullptr;        // device, >= radix_count_words(S, max_seg_len)
    int begin_bit = 0;
    int end_bit = 64;
    Profiler* prof = nullptr;          // optional
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per workgroup tile

// Which key range a workgroup tile covers.  Fixed mode (tile_seg == nullptr):
// segment s owns tiles [s*tps, (s+1)*tps).  List mode: tile i belongs to
// segment tile_seg[i], whose tiles are [tile0[s], tile0[s+1]).  Segment s
// spans [beg[s], end[s]).
struct TileMap {
    const uint64_t* beg = nullptr;
    const uint64_t* end = nullptr;
    // optional per-segment key offset: digits are taken from key - base[s]
    const uint64_t* base = nullptr;
    const uint32_t* tile_seg = nullptr;
    const uint32_t* tile0 = nullptr;
    uint32_t tps = 0;
};

// One stable counting pass on digit [shift, shift+8) of every segment.
struct RadixPass {
    int key_bytes = 8;
    const void* keys_in = nullptr;
    const uint64_t* vals_in = nullptr;
    void* keys_out = nullptr;
    uint64_t* vals_out = nullptr;
    TileMap map;
    uint32_t num_segs = 0;
    uint32_t num_tiles = 0;
    int shift = 0;
    const uint8_t* seg_shift = nullptr;  // optional: per-segment digit shift (fixed mode)
    uint32_t* counts = nullptr;        // num_tiles * 256 words
    uint64_t* sb_start = nullptr;      // optional: per (segment, digit) run start
    uint32_t* sb_len = nullptr;        // optional: per (segment, digit) run length
    uint64_t total_len = 0;            // keys covered (for byte counts)
    // keys only and the order of equal digits within a run is free (a pass
    // whose runs are fully sorted afterwards): rank by LDS atomics
    bool any_order = false;
    Profiler* prof = nullptr;
};

uint64_t radix_count_words(uint32_t num_segs, uint64_t max_seg_len);
hipError_t radix_pass(const RadixPass& a, hipStream_t stream);
hipError_t segmented_radix_sort(const SegSort& a, hipStream_t stream);

// --------------------------------------------------------------- fences ----
// Every kFenceStride-th key of each locally sorted segment, kept so that a
// search inside a segment can start from on-chip fences and finish inside
// one cache line: key[s * per_seg + f] = key at position f * kFenceStride of
// segment s (widened to 64 bits).
constexpr int kFenceStride = 16;

struct Fences {
    uint64_t* key = nullptr;
    uint64_t per_seg = 0;              // ceil(max segment length / kFenceStride)
};

// ---------------------------------------------------------- hybrid sort ----
// Sub-buckets too large for LDS, collected on the device.
struct OversizeList {
    uint32_t* count = nullptr;         // entries
    uint32_t* tiles = nullptr;         // total tiles
    uint64_t* beg = nullptr;           // capacity oversize_capacity()
    uint64_t* end = nullptr;
    uint64_t* base = nullptr;          // key offset of the entry's segment
    uint32_t* seg = nullptr;           // segment of the entry
    uint32_t* tile0 = nullptr;         // capacity + 1
    uint32_t* tile_seg = nullptr;      // oversize_tile_capacity()
    uint32_t* summary = nullptr;       // 4 words for the host: entries, tiles, slow-list entries
};

// Sub-buckets that fit LDS but hold a large group of keys equal in their
// next 8 bits, collected on the device for the LDS-LSD kernel.
struct SlowList {
    uint32_t* count = nullptr;
    uint64_t* beg = nullptr;           // capacity slow_capacity()
    uint32_t* len = nullptr;
    uint8_t* bits = nullptr;           // bits of key - base below which keys still differ
    uint64_t* base = nullptr;          // key offset of the entry's segment
    uint32_t* seg = nullptr;           // segment of the entry
};

// Stable sort of contiguous segments [seg_off[s], seg_off[s+1]): an MSD pass
// into keys_tmp, then every sub-bucket finished into keys_out.  keys_in must
// differ from keys_tmp and keys_out.
struct HybridSort {
    int key_bytes = 8;
    const void* keys_in = nullptr;
    const uint64_t* vals_in = nullptr;
    void* keys_out = nullptr;
    uint64_t* vals_out = nullptr;
    void* keys_tmp = nullptr;
    uint64_t* vals_tmp = nullptr;
    const uint64_t* seg_off = nullptr;
    uint32_t num_segs = 0;
    uint64_t max_seg_len = 0;
    uint64_t total_len = 0;
    uint32_t* counts = nullptr;        // >= radix_count_words(num_segs, max_seg_len)
    uint64_t* sb_start = nullptr;      // num_segs * 256
    uint32_t* sb_len = nullptr;        // num_segs * 256
    // optional per-segment MSD digit: every key k of segment s must satisfy
    // 0 <= k - seg_base[s] < 2^(seg_shift[s] + 8); the MSD digit is then
    // (k - seg_base[s]) >> seg_shift[s].  nullptr: base 0, the top digit.
    const uint8_t* seg_shift = nullptr;
    const uint64_t* seg_base = nullptr;
    OversizeList ov;
    SlowList sl;
    Fences fences;                     // optional: written for the sorted output
    Profiler* prof = nullptr;
};

// Host-side state of the hybrid sort: pinned read-back words and the count
// table of the oversize passes, grown on demand.
struct HybridHost {
    uint32_t* pinned = nullptr;        // 4 words
    uint32_t* fb_counts = nullptr;
    uint64_t fb_words = 0;
    uint32_t last_oversize = 0;
    uint32_t last_slow = 0;
};

hipError_t hybrid_sort(const HybridSort& a, hipStream_t s, HybridHost& host);
uint64_t oversize_capacity(uint32_t num_segs, uint64_t total_len);
uint64_t oversize_tile_capacity(uint32_t num_segs, uint64_t total_len);
uint64_t slow_capacity(uint32_t num_segs, uint64_t total_len);

// --------------------------------------------------------------- rounds ----
// Device counters read back once per round.
struct RoundCounters {
    unsigned long long m;          // probes emitted this round (may exceed capacity)
    unsigned long long domain;     // keys in the sampled domain
    unsigned long long blocks;     // Philox blocks in the flattened domain
    unsigned int n_ivl;            // distinct unsettled intervals
    unsigned int n_slices;         // non-empty (interval, segment) slices
    unsigned int n_unsettled;      // unsettled splitters before the round
    unsigned int n_req;            // locate requests emitted by the settle step
    unsigned int err;              // device consistency failures (bit set)
};

enum DeviceErr : unsigned int {
    kErrProbeOutside = 1u,         // a probe outside its own interval slice
    kErrRankOrder = 2u,            // ranks not strictly increasing in probe order
    kErrPieceSum = 4u,             // bucket pieces do not add up to the bucket size
};

struct RoundArgs {
    int key_bytes;
    const void* B;                 // locally sorted keys
    uint64_t n;
    uint32_t p;
    const uint64_t* seg_off;       // p+1
    const uint64_t* ideal;         // p+1, floor(i N / p)
    uint64_t tol;
    // splitter state, indexed 0..p (1..p-1 used)
    uint32_t* settled;
    uint64_t* chi;
    uint64_t* lrank;
    uint64_t* urank;
    uint64_t* s_key;
    uint64_t* s_tag;
    uint32_t* lpos;                // (p+1) x p
    uint32_t* upos;                // (p+1) x p
    uint32_t* prow;                // (p+1) x p
    // intervals
    uint32_t* ivl_row;             // p
    uint4* slices;                 // p x p: non-empty slices {first block, first tag, end tag, interval}
    uint32_t* ivl_nz;              // p+1: non-empty slice counts, then exclusive offsets
    uint64_t* ivl_tot;             // p+1: block totals, then exclusive offsets
    uint64_t* ivl_dom;             // p
    // probes
    uint64_t cap;                  // probe capacity
    uint64_t* pr_key;
    uint64_t* pr_tag;
    uint32_t* pr_ivl;
    uint64_t* ps_key;              // sorted
    uint64_t* ps_tag;
    uint32_t* ps_ivl;
    uint64_t* pr_rank;             // rank R of sorted probe e
    uint32_t* pr_pos;              // sorted position of emitted probe
    uint32_t* ps_seg;              // segment of sorted probe e
    // requests
    uint32_t* req_probe;
    uint32_t* req_row;
    uint32_t* req_kind;
    RoundCounters* ctr;
};

hipError_t launch_round_init(const RoundArgs& a, hipStream_t s);
// Zero the round counters (the device error word included).
hipError_t launch_counters_reset(RoundCounters* ctr, hipStream_t s);
hipError_t launch_intervals(const RoundArgs& a, hipStream_t s);
hipError_t launch_sample(const RoundArgs& a, uint64_t seed, uint32_t round, uint32_t thresh,
                         int take_all, hipStream_t s);
// Sort the m emitted probes by (key, tag) into ps_*; uses sort scratch for
// large m.
hipError_t launch_probe_sort(const RoundArgs& a, uint64_t m, void* scratch, size_t scratch_bytes,
                             uint32_t* counts, hipStream_t s);
size_t probe_sort_scratch_bytes(uint64_t m);
// cmat (optional, p x m words, segment-major): c_s(e) at cmat[s * m + e],
// kept for locate.  With fences (and cmat), the counts are found per
// (segment, chunk) from on-chip fences; otherwise per probe by searching
// every segment's slice.
hipError_t launch_rank(const RoundArgs& a, uint64_t m, uint32_t* cmat, const Fences& fences,
                       uint64_t max_seg, hipStream_t s);
hipError_t launch_settle(const RoundArgs& a, uint64_t m, hipStream_t s);
hipError_t launch_locate(const RoundArgs& a, const uint32_t* cmat, uint64_t m, hipStream_t s);
hipError_t launch_finalize(const RoundArgs& a, uint64_t* d_offsets, hipStream_t s);

// ------------------------------------------------------------- exchange ----
struct ExchangeArgs {
    int key_bytes;
    const void* B;
    const uint64_t* Bv;            // nullptr: keys only
    void* out;
    uint64_t* vout;
    uint64_t n;
    uint32_t p;
    const uint64_t* seg_off;       // p+1
    const uint32_t* prow;          // (p+1) x p, rows 1..p-1 used
    const uint64_t* chi;           // p+1 (the offsets array)
    uint32_t* dst;                 // p x p, offset of piece (b, s) inside bucket b
    uint64_t max_bucket;
    unsigned int* err;
    Profiler* prof = nullptr;      // optional
};

hipError_t launch_exchange(const ExchangeArgs& a, hipStream_t s);
// Per-bucket MSD digit for the bucket sort: all keys of bucket b lie in
// [lo, hi] = [key(S(b)), key(S(b+1))] (0 and the largest key at the ends), so
// with base = lo the offsets key - lo fit below 2^(shift + 8) for the
// smallest shift with hi - lo < 2^(shift + 8).
hipError_t launch_bucket_shift(uint32_t p, int key_bits, const uint64_t* s_key, uint8_t* shift,
                               uint64_t* base, hipStream_t s);

}  // namespace hss
