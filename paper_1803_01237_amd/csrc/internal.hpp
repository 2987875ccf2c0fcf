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
    // optional per-segment source: device addresses of the segment's first
    // key (and payload word); otherwise the pass input at position beg[s]
    const uint64_t* src = nullptr;
    const uint64_t* vsrc = nullptr;
    // optional per-segment destination: device addresses where the
    // segment's first key (and payload word) go; otherwise the pass output at
    // position beg[s]
    const uint64_t* dst = nullptr;
    const uint64_t* vdst = nullptr;
    // optional: segments flagged here are left alone by the scatter
    const uint8_t* skip = nullptr;
    // optional (splitter levels): per-segment tables of kSplitSlots keys,
    // n_splits[s] splitters ascending then all ones; a key's "digit" is its
    // class among them (2 j + 1: equal to splitter j; 2 j: between splitters
    // j - 1 and j)
    const uint64_t* splits = nullptr;
    const uint32_t* n_splits = nullptr;
};

// Splitter table of one entry of a splitter level: at most kSplitSlots - 1
// splitters, so that classes 0 .. 2 (kSplitSlots - 1) fit 256 digits.
constexpr uint32_t kSplitSlots = 128;

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
    bool has_payload = false;          // payload read through map.vsrc (vals_in may be null)
    // optional per-segment AND and OR of every key - base (the bits that
    // vary inside the segment), accumulated by the count pass; both must be
    // preset to all ones and zero
    uint64_t* and_mask = nullptr;
    uint64_t* or_mask = nullptr;
    // the counts (and masks) were already taken by the kernel that wrote the
    // keys: the pass only scans them
    bool counted = false;
    Profiler* prof = nullptr;
};

uint64_t radix_count_words(uint32_t num_segs, uint64_t max_seg_len);
hipError_t radix_pass(const RadixPass& a, hipStream_t stream);
// The pass in two halves (count and scan; scatter), for work in between.
hipError_t radix_count_scan(const RadixPass& a, hipStream_t stream);
hipError_t radix_scatter(const RadixPass& a, hipStream_t stream);
hipError_t segmented_radix_sort(const SegSort& a, hipStream_t stream);

// --------------------------------------------------------------- fences ----
// Every kFenceStride-th key of each locally sorted segment, kept so that a
// search inside a segment can start from on-chip fences and finish inside
// one cache line: key[base[s] + f] = key at position f * kFenceStride of
// segment s (widened to 64 bits); base[s] = sum over earlier segments of
// ceil(length / kFenceStride).
constexpr int kFenceStride = 16;

struct Fences {
    uint64_t* key = nullptr;
    const uint64_t* base = nullptr;    // S+1 entries
    const uint64_t* seg_off = nullptr; // S+1 entries, positions of the sorted buffer
};

// Fences of segments sorted by another path (the LSD-only mode).
hipError_t write_fences(const void* keys, int key_bytes, uint32_t num_segs, const Fences& f,
                        hipStream_t s);

// ---------------------------------------------------------- hybrid sort ----
// Sub-buckets too large for LDS, collected on the device.
// Where the keys of a pending range are: the MSD buffer, the output, or the
// sort's input (a segment whose top digit held all its keys).
enum : uint8_t { kLocTmp = 0, kLocOut = 1, kLocIn = 2 };

// Key ranges still to sort after a level of MSD passes: sub-buckets above the
// small-sort capacity, and ranges whose digit held every key (retried on the
// highest bit that varies).  Every key k of an entry satisfies k - base <
// 2^bits; its keys sit at src (payload vsrc) in buffer `loc`.
struct OversizeList {
    uint32_t* count = nullptr;         // entries
    uint32_t* tiles = nullptr;         // total tiles
    uint64_t* beg = nullptr;           // capacity oversize_capacity()
    uint64_t* end = nullptr;
    uint64_t* base = nullptr;          // key offset of the entry's segment
    uint32_t* seg = nullptr;           // segment of the entry
    uint8_t* bits = nullptr;
    uint8_t* loc = nullptr;
    uint64_t* src = nullptr;           // device address of the entry's first key
    uint64_t* vsrc = nullptr;          // and payload word
    uint32_t* tile0 = nullptr;         // capacity + 1
    uint32_t* tile_seg = nullptr;      // oversize_tile_capacity()
    uint32_t* summary = nullptr;       // 5 words for the host: entries, tiles, slow-list
                                       // and equal-list entries, overrun flag
    uint32_t capacity = 0;
    uint32_t* err = nullptr;           // set when a push finds the list full
};

// Ranges whose keys are all equal: already sorted, copied to the output
// (unless there) and given their fences at the end of the sort.
struct EqualList {
    uint32_t* count = nullptr;
    uint64_t* beg = nullptr;           // capacity oversize_capacity()
    uint64_t* end = nullptr;
    uint32_t* seg = nullptr;
    uint8_t* loc = nullptr;
    uint64_t* src = nullptr;
    uint64_t* vsrc = nullptr;
    uint32_t capacity = 0;
    uint32_t* err = nullptr;
};

// Small-sort jobs of a deeper level: runs of consecutive sub-buckets of one
// entry packed up to the small-sort capacity (a sub-bucket above it is a job
// of its own and goes on to the next level).  Capacity packed_capacity().
struct PackedJobs {
    uint32_t* count = nullptr;
    uint64_t* start = nullptr;         // first position
    uint32_t* len = nullptr;
    uint32_t* entry = nullptr;         // entry of the level's list
    uint64_t* base = nullptr;          // key offset of the job: entry base + first digit
    uint8_t* bits = nullptr;           // free bits of key - base inside the job
    uint32_t capacity = 0;
    uint32_t* err = nullptr;
    // Staging: entry e writes its jobs at slots from stage_slot(e) (room for
    // the at most 8 jobs per tile of 4096 keys plus one it can give) and
    // their number in n_of[e]; a scan over the entries then packs them into
    // the arrays above.  No counter is shared between entries: one atomic
    // per entry on one word would take its turn with every other entry's.
    uint64_t* s_start = nullptr;       // capacity stage_capacity()
    uint32_t* s_len = nullptr;
    uint64_t* s_base = nullptr;
    uint8_t* s_bits = nullptr;
    uint64_t s_capacity = 0;
    uint32_t* n_of = nullptr;          // level_capacity() + 1
    uint32_t* chunk_sum = nullptr;     // level_capacity() / kPackChunk + 2
};
constexpr uint32_t kPackChunk = 1024;  // entries per workgroup of the packing

// Per-entry work arrays of one MSD level (level 1: the MSD segments; deeper:
// the entries of an OversizeList), capacity level_capacity().
struct LevelWork {
    uint8_t* shift = nullptr;          // digit [shift, shift + 8) of key - base
    uint8_t* skip = nullptr;           // 1: the digit held every key, no scatter
    uint64_t* dst = nullptr;           // where the scatter writes the entry
    uint64_t* vdst = nullptr;
    uint64_t* and_mask = nullptr;
    uint64_t* or_mask = nullptr;
    uint64_t* splits = nullptr;        // kSplitSlots keys per entry of a level
    uint32_t* n_splits = nullptr;      // splitters of every entry
    uint32_t* split_entries = nullptr; // nonzero when an entry of the level has splitters
};

// Sub-buckets that fit LDS but hold a large group of keys equal in their
// next bits, collected on the device for the slow-path kernel.
struct SlowList {
    uint32_t* count = nullptr;
    uint64_t* beg = nullptr;           // capacity slow_capacity()
    uint32_t* len = nullptr;
    uint32_t* seg = nullptr;           // segment of the entry
    uint32_t capacity = 0;
    uint32_t* err = nullptr;
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
    uint64_t min_seg_len = 0;          // shortest segment of the first level (0: not known)
    uint64_t max_seg_len = 0;
    uint64_t total_len = 0;
    uint32_t* counts = nullptr;        // >= radix_count_words(num_segs, max_seg_len)
    uint64_t* sb_start = nullptr;      // num_segs * 256
    uint32_t* sb_len = nullptr;        // num_segs * 256
    // optional MSD digit per entry of the MSD pass (segment s, or list entry
    // s when msd_seg is given): every key k of the entry must satisfy
    // 0 <= k - seg_base[s] < 2^(seg_shift[s] + 8); the MSD digit is then
    // (k - seg_base[s]) >> seg_shift[s].  nullptr: base 0, the top digit.
    const uint8_t* seg_shift = nullptr;
    const uint64_t* seg_base = nullptr;
    // the first level's digit counts per 4096-key tile and the segments'
    // AND/OR masks were taken while the keys were written (counts laid out as
    // the count pass would, every tile past a segment's end zero)
    bool counted = false;
    OversizeList ov;                   // two lists, alternating between levels
    OversizeList ov2;
    EqualList eq;
    LevelWork lw;
    PackedJobs pj;
    SlowList sl;
    Fences fences;                     // optional: written for the sorted output
    Profiler* prof = nullptr;
    // Segment selection (all optional).  By default every segment s of
    // seg_off takes the MSD pass.  With msd_seg, only the listed segments do
    // (num_segs of them, spanning [msd_beg[i], msd_end[i]) with the tile list
    // msd_tile_seg / msd_tile0 of msd_tiles tiles), and the n_direct
    // segments of direct_seg (at most the small-sort capacity each) are
    // sorted in one step.  msd_src / direct_src give per-segment device
    // addresses of the input keys (payload: *_vsrc); otherwise keys_in at
    // the segment's position.
    bool has_payload = false;          // payload read through the *_vsrc sources
    bool cap_large = false;            // on-chip jobs of 4096 keys (else 2048; 4096 always
                                       // with seg_base)
    const uint32_t* msd_seg = nullptr;
    const uint64_t* msd_beg = nullptr;
    const uint64_t* msd_end = nullptr;
    const uint32_t* msd_tile_seg = nullptr;
    const uint32_t* msd_tile0 = nullptr;
    uint32_t msd_tiles = 0;
    const uint64_t* msd_src = nullptr;
    const uint64_t* msd_vsrc = nullptr;
    const uint32_t* direct_seg = nullptr;
    uint32_t n_direct = 0;
    const uint64_t* direct_src = nullptr;
    const uint64_t* direct_vsrc = nullptr;
};

// Largest segment the small sort takes in one step (direct segments).
constexpr uint32_t kDirectSegMax = 2048;

// Device and pinned host memory of an engine: hipMalloc / hipHostMalloc by
// default, or a cache of blocks kept between the batches of a server.
struct MemSource {
    virtual hipError_t dev_get(void** p, size_t bytes) = 0;
    virtual void dev_put(void* p) = 0;
    virtual hipError_t host_get(void** p, size_t bytes) = 0;
    virtual void host_put(void* p) = 0;
    virtual ~MemSource() = default;
};
// With m null: hipMalloc / hipFree, hipHostMalloc / hipHostFree.
hipError_t dev_alloc(MemSource* m, void** p, size_t bytes);
void dev_release(MemSource* m, void* p);
hipError_t host_alloc(MemSource* m, void** p, size_t bytes);
void host_release(MemSource* m, void* p);

// Host-side state of the hybrid sort: pinned read-back words and the count
// table of the oversize passes, grown on demand.
struct HybridHost {
    uint32_t* pinned = nullptr;        // 8 words
    uint32_t* fb_counts = nullptr;     // count table of the deeper levels
    uint64_t fb_words = 0;
    uint64_t* fb_sb_start = nullptr;   // their sub-bucket tables
    uint32_t* fb_sb_len = nullptr;
    uint64_t fb_sb = 0;
    MemSource* mem = nullptr;          // where the grown tables come from
    uint32_t last_oversize = 0;        // entries of the first deeper level
    uint32_t last_slow = 0;
    uint32_t last_levels = 0;          // deeper levels run
    // the first level's splitter flag: waited for through this event (the
    // count by digits queued behind its copy), unless the last call took
    // splitters there; null: the stream is waited for
    hipEvent_t flag_ev = nullptr;
    bool split1_last = false;
};

hipError_t hybrid_sort(const HybridSort& a, hipStream_t s, HybridHost& host);
// List capacities: every list holds disjoint key ranges above a size, so the
// bounds follow from the number of keys alone.
uint64_t oversize_capacity(uint64_t total_len);
uint64_t oversize_tile_capacity(uint64_t total_len);
uint64_t level_capacity(uint32_t num_segs, uint64_t total_len);
uint64_t packed_capacity(uint64_t total_len);
uint64_t stage_capacity(uint32_t num_segs, uint64_t total_len);
uint64_t slow_capacity(uint64_t total_len);

// --------------------------------------------------------------- rounds ----
// The splitter rounds of any number of independent instances at once.  Index
// spaces (all global over the instances of a plan):
//   positions  instance I owns [pos0, pos0 + n) of the sorted buffer B; its
//              tags g (section 6.1) are positions relative to pos0
//   segments   instance I owns segments [seg0, seg0 + p)
//   rows       instance I owns splitter rows [row0, row0 + p]; row row0 + i
//              holds splitter i (rows i = 0 and i = p are the fixed ends)
//   tables     per-segment counts of instance I's row i live at
//              tab0 + i * p + s, s < p (lpos, upos, prow)
struct InstDesc {
    uint64_t n;
    uint64_t pos0;
    uint64_t tol;
    uint64_t tab0;
    uint32_t p;                    // segments (virtual processors)
    uint32_t seg0;
    uint32_t row0;                 // rows: splitters 0..q
    uint32_t q;                    // buckets (= p, or fewer: a stage of multi-stage HSS)
};

// Per call: seed and the caller's buffers of every instance.
struct InstRun {
    uint64_t seed;
    const void* kin;
    const uint64_t* vin;
    void* kout;
    uint64_t* vout;
    uint64_t* offsets;             // p + 1 entries: chi
};

// Device counters of the current round and of the call.
struct RoundCounters {
    unsigned long long m;          // probes emitted this round (may exceed capacity)
    unsigned long long domain;     // tags in the sampled domain
    unsigned long long blocks;     // Philox blocks in the flattened domain
    unsigned long long m_stored;   // probes kept (m unless over capacity)
    unsigned long long cm_need;    // count-matrix words of this round
    unsigned long long m_max;      // largest m of the call (capacity growth)
    unsigned long long cm_max;     // largest cm_need of the call
    unsigned int n_ivl;            // distinct unsettled intervals
    unsigned int n_slices;         // non-empty (interval, segment) slices
    unsigned int n_unsettled;      // unsettled splitters before the round
    unsigned int n_after;          // unsettled splitters after the round
    unsigned int tiles;            // workgroups of the probe ranking
    unsigned int err;              // device consistency failures (bit set)
    unsigned int overflow;         // a capacity was exceeded: the call's later work is skipped
};

// Counts of round j, kept for the host to read once after the rounds.
struct RoundHist {
    unsigned long long domain;     // tags sampled from
    unsigned long long m;          // probes
    unsigned int unsettled;        // unsettled splitters before the round
    unsigned int thresh;           // acceptance threshold of instance 0
    unsigned int all;              // 1: every tag of the domain was a probe
    unsigned int pad;
};

enum DeviceErr : unsigned int {
    kErrProbeOutside = 1u,         // a probe outside its own interval slice
    kErrRankOrder = 2u,            // ranks not strictly increasing in probe order
    kErrPieceSum = 4u,             // a bucket's pieces do not add up to chi(b+1) - chi(b)
};

// Rounds whose draws may be taken ahead.  The draws of a round cost about
// 0.25 ms of ALU work at 2^28 keys; two rounds fit beside the count pass of
// the local sort (a pure stream), more spill into the scatter and slow it.
constexpr uint32_t kPreRounds = 2;

struct RoundArgs {
    int key_bytes;
    const void* B;                 // locally sorted keys of all instances
    uint32_t n_inst, n_rows, n_segs, p_max;
    uint32_t J;                    // rounds in the rate table
    const InstDesc* inst;
    const InstRun* run;
    uint32_t* thresh;              // n_inst x J: acceptance threshold of round j at [I J + j - 1]
    uint8_t* all;                  // n_inst x J: 1 = every tag of the domain is a probe
    uint32_t budget;               // c > 0: rate c p / |gamma| set on the device each round
                                   // (one instance)
    uint32_t picks;                // 1 (with a budget c): section 6's sampler, ceil(c N /
                                   // |gamma|) picks of every segment per round, kept when
                                   // inside an interval (one instance); the round's
                                   // threshold is the pick count
    uint32_t* pick_bits;           // picks: one bit per tag, set by a kept pick (each
                                   // position kept once); cleared after every round
    uint64_t pick_words;           // words of pick_bits
    uint32_t pair_rank_from;       // first round ranked per (probe, segment) pair inside
                                   // the probe's interval slice (earlier: by segment chunks)
    uint32_t sample_grid;          // workgroups of the sampler
    uint32_t pair_grid;            // workgroups of the per-pair rank search
    uint32_t dense_rank;           // 1: round 1 ranks its probes against the chunk's keys
                                   // staged in LDS (probes denser than the fences)
    // one instance: the draws of rounds 1..kPreRounds taken ahead of the
    // rounds: pre_list[j-1] holds, in any order, every tag whose Philox word
    // of round j is below the round's threshold (pre_cnt[j-1] of them; more
    // than pre_cap: the list is incomplete and the sampler draws itself), or
    // null
    const uint32_t* pre_list[kPreRounds];
    const uint32_t* pre_cnt[kPreRounds];
    uint32_t pre_cap;
    const uint64_t* seg_off;       // S+1 positions
    const uint32_t* seg_inst;      // S
    const uint32_t* row_inst;      // Q
    const uint64_t* ideal;         // Q: floor(i n / p) of row i
    // splitter state, Q rows
    uint32_t* settled;
    uint64_t* chi;
    uint64_t* lrank;
    uint64_t* urank;
    uint64_t* s_key;
    uint64_t* s_tag;
    uint64_t* l_tag;               // tags of the probes at the bounds L and U (when set)
    uint64_t* u_tag;
    uint32_t* lpos;                // sum over instances of (p+1) p
    uint32_t* upos;
    uint32_t* prow;
    // intervals (at most Q)
    uint32_t* ivl_row;
    uint32_t* ivl_inst;
    uint64_t* ivl_tot;             // Philox blocks, then exclusive offsets
    uint32_t* ivl_nz;              // non-empty slices, then exclusive offsets
    uint64_t* ivl_dom;
    uint32_t* ivl_pcnt;            // probes of the interval
    uint32_t* ivl_poff;            // their first sorted index
    uint32_t* ivl_cursor;
    uint32_t* ivl_tile0;           // first ranking workgroup of the interval
    // the interval's bounds in the order (key, tag): keys as unsigned, tags
    // as signed; an open end is (0, -1) below and (all ones, INT64_MAX) above
    uint64_t* ivl_lkey;
    int64_t* ivl_ltag;
    uint64_t* ivl_ukey;
    int64_t* ivl_utag;
    uint4* slices;                 // {first block, first tag, end tag, interval}
    // per instance, per round
    uint32_t* inst_plo;            // first sorted probe of the instance
    uint32_t* inst_pm;             // its probes
    uint64_t* cm_off;              // its count-matrix block
    // per splitter row, two slots of probes whose per-segment counts become
    // table rows: slot 2r the new lower bound (or the settling probe), slot
    // 2r+1 the new upper bound; sel_e = sorted probe index or kNoSel
    uint32_t* sel_e;
    uint8_t* sel_kind;             // 0: lpos, 1: upos, 2: prow
    // probes (capacity cap)
    uint64_t cap;
    uint64_t* pr_key;
    uint64_t* pr_tag;
    uint32_t* pr_ivl;
    uint64_t* g_key;               // grouped by interval
    uint64_t* g_tag;
    uint64_t* ps_key;              // sorted by (instance, key, tag)
    uint64_t* ps_tag;
    uint32_t* ps_ivl;
    uint32_t* ps_seg;
    uint32_t* ps_row;              // the interval's splitter row, with kRowLNone / kRowUNone
    uint64_t* pr_rank;
    uint32_t* cmat;                // count matrix, capacity cm_cap words
    uint64_t cm_cap;
    // rank work list: chunk c covers keys [chunk_lo[c], +kRankChunk) of segment chunk_seg[c]
    const uint32_t* chunk_seg;
    const uint32_t* chunk_lo;
    uint32_t n_chunks;
    Fences fences;                 // of B
    RoundCounters* ctr;
    RoundHist* hist;               // J entries
};

constexpr uint32_t kRankChunk = 1u << 15;   // keys of a segment per rank workgroup
constexpr uint32_t kNoSel = 0xFFFFFFFFu;    // empty selection slot
// Flags of a sorted probe's splitter row (ps_row): the interval is open below
// (L = -infinity) or above (U = +infinity); rows are below 2^30.
constexpr uint32_t kRowLNone = 1u << 31;
constexpr uint32_t kRowUNone = 1u << 30;
constexpr uint32_t kRowMask = kRowUNone - 1;

hipError_t launch_counters_reset(RoundCounters* ctr, hipStream_t s);
// Start of a call's rounds: every splitter unsettled with open bounds.
// Every tag g < n whose Philox word of round `round` is below `thresh` (the
// sampler's decision, which does not depend on the keys), appended in any
// order to list (capacity cap; *count receives the full number).
hipError_t launch_presample(uint64_t seed, uint64_t n, uint32_t round, uint32_t thresh, uint32_t* list,
                            uint32_t cap, uint32_t* count, hipStream_t s);
hipError_t launch_presample_reset(uint32_t* counts, uint32_t n, hipStream_t s);
hipError_t launch_round_init(const RoundArgs& a, hipStream_t s);
// One whole round j (section 4.2.2 steps 1-5) for every instance; sizes are
// read on the device, so nothing here waits for the host.
hipError_t launch_round(const RoundArgs& a, uint32_t j, hipStream_t s, Profiler* prof);
// chi of every instance into its offsets array and into chi_all (Q entries).
hipError_t launch_finalize(const RoundArgs& a, uint64_t* chi_all, hipStream_t s);
// A round in two halves: intervals, sampling, probe offsets and grouping by
// interval (g_key, g_tag); then ordering (skipped when the caller has put
// every interval's probes in (key, tag) order into ps_key / ps_tag and run
// launch_probe_finish), ranks, reduction and settling.
hipError_t launch_round_head(const RoundArgs& a, uint32_t j, hipStream_t s);
hipError_t launch_round_tail(const RoundArgs& a, uint32_t j, hipStream_t s, bool probes_sorted,
                             Profiler* prof);
hipError_t launch_probe_offsets(const RoundArgs& a, uint64_t* out, hipStream_t s);
hipError_t launch_probe_finish(const RoundArgs& a, hipStream_t s);
// The per-call record of one instance, written on the stream (no host copy).
hipError_t launch_set_run(const InstRun& r, InstRun* dst, hipStream_t s);
// Caller buffers per segment: device addresses of the input keys (and
// payload) of the segments list[x] (x < count; nullptr: segment x) for the
// first sort pass.
hipError_t launch_segment_sources(const RoundArgs& a, const uint32_t* list, uint32_t count,
                                  uint64_t* key_src, uint64_t* val_src, int key_bytes,
                                  hipStream_t s);

// ------------------------------------------------------------- exchange ----
struct ExchangeArgs {
    int key_bytes;
    const void* B;                 // locally sorted keys of all instances
    const uint64_t* Bv;            // nullptr: keys only
    uint32_t n_inst;
    uint32_t n_rows;               // rows of all instances: bucket b of instance I is row
                                   // row0 + b (the last row of an instance is no bucket)
    uint32_t p_max;                // largest p of the instances
    const InstDesc* inst;
    const InstRun* run;
    const uint64_t* seg_off;
    const uint32_t* row_inst;
    const uint32_t* prow;
    const uint64_t* chi_all;       // Q rows
    uint32_t* dst;                 // table-shaped: offset of piece (b, s) inside bucket b
    uint32_t* chunk0;              // Q+1: first copy workgroup of every bucket (row)
    uint64_t max_chunks;           // bound on the copy workgroups
    uint64_t total;                // keys of all instances
    // one instance, before its bucket sort: each copy workgroup also counts
    // the digits ((key - base[b]) >> shift[b]) & 255 of its 4096 outputs (the
    // bucket's tile) into counts[(b tps + tile) 256 + digit], and the AND and
    // OR of key - base[b] into and_mask[b], or_mask[b]; null: no counting
    uint32_t* sort_counts = nullptr;
    uint32_t sort_tps = 0;
    const uint8_t* sort_shift = nullptr;
    const uint64_t* sort_base = nullptr;
    uint64_t* sort_and = nullptr;
    uint64_t* sort_or = nullptr;
    // output: the caller's buffers of every instance, or (when out is set)
    // one buffer at the instance positions
    void* out = nullptr;
    uint64_t* vout = nullptr;
    unsigned int* err;
    Profiler* prof = nullptr;      // optional
    // when set, every kernel does nothing unless the rounds before it left
    // no splitter unsettled and no buffer overrun (rounds queued ahead of
    // their read-back)
    const RoundCounters* gate = nullptr;
};

hipError_t launch_exchange(const ExchangeArgs& a, hipStream_t s);
// out[g pg + i] = chi1[g] + off2[g (pg+1) + i] for g < r, i < pg; out[r pg] = n.
// Key range of every MSD list entry of a multi-instance engine from the range
// of its instance: shift[li] = ishift[I], base[li] = ibase[I] with
// I = seg_inst[msd_seg[li]].
hipError_t launch_entry_ranges(uint32_t n_msd, const uint32_t* msd_seg, const uint32_t* seg_inst,
                               const uint8_t* ishift, const uint64_t* ibase, uint8_t* shift,
                               uint64_t* base, hipStream_t s);
// The bucket sort's first level counted by the exchange: zero the count
// table (words) and preset the n masks.
hipError_t launch_sort_count_reset(uint32_t* counts, uint64_t words, LevelWork w, uint32_t n, hipStream_t s);
hipError_t launch_stage_offsets(const uint64_t* chi1, const uint64_t* off2, uint32_t r, uint32_t pg,
                                uint64_t n, uint64_t* out, hipStream_t s);
// Per-bucket MSD digit for the bucket sort: all keys of bucket b lie in
// [lo, hi] = [key(S(b)), key(S(b+1))] (0 and the largest key at the ends), so
// with base = lo the offsets key - lo fit below 2^(shift + 8) for the
// smallest shift with hi - lo < 2^(shift + 8).
hipError_t launch_bucket_shift(uint32_t p, int key_bits, const uint64_t* s_key, uint8_t* shift,
                               uint64_t* base, hipStream_t s);
// Upper bound of the copy workgroups for buckets of at most `total` keys.
uint64_t exchange_chunk_bound(uint64_t total, uint32_t buckets);

}  // namespace hss
