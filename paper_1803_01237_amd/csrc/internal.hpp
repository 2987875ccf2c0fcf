// Host-side interfaces between the executor (hss.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hss {

constexpr uint64_t kNone = ~0ull;

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
    uint32_t* counts = nullptr;        // device, >= radix_count_words(S, max_seg_len)
    int begin_bit = 0;
    int end_bit = 64;
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;   // keys per workgroup tile

uint64_t radix_count_words(uint32_t num_segs, uint64_t max_seg_len);
hipError_t segmented_radix_sort(const SegSort& a, hipStream_t stream);

// --------------------------------------------------------------- rounds ----
// Device counters read back once per round.
struct RoundCounters {
    unsigned long long m;          // probes emitted this round (may exceed capacity)
    unsigned long long domain;     // keys in the sampled domain
    unsigned long long blocks;     // Philox blocks in the flattened domain
    unsigned int n_ivl;            // distinct unsettled intervals
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
    uint32_t* ivl_blk;             // p x p, exclusive block offset of slice (k, s) in interval k
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
    // requests
    uint32_t* req_probe;
    uint32_t* req_row;
    uint32_t* req_kind;
    RoundCounters* ctr;
};

hipError_t launch_round_init(const RoundArgs& a, hipStream_t s);
hipError_t launch_intervals(const RoundArgs& a, hipStream_t s);
hipError_t launch_sample(const RoundArgs& a, uint64_t seed, uint32_t round, uint32_t thresh,
                         int take_all, hipStream_t s);
// Sort the m emitted probes by (key, tag) into ps_*; uses sort scratch for
// large m.
hipError_t launch_probe_sort(const RoundArgs& a, uint64_t m, void* scratch, size_t scratch_bytes,
                             uint32_t* counts, hipStream_t s);
size_t probe_sort_scratch_bytes(uint64_t m);
hipError_t launch_rank(const RoundArgs& a, uint64_t m, hipStream_t s);
hipError_t launch_settle(const RoundArgs& a, uint64_t m, hipStream_t s);
hipError_t launch_locate(const RoundArgs& a, hipStream_t s);
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
};

hipError_t launch_exchange(const ExchangeArgs& a, hipStream_t s);

}  // namespace hss
