// libhss: plans, executor and C ABI of Histogram Sort with Sampling on one
// device.  An engine holds one or more independent instances with the same
// key type; every phase (local sort, splitter rounds, exchange) runs all of
// them in the same launches.  hss_plan is an engine of one instance;
// hss_batch_plan groups a list of instances into one engine per key type.
// The splitter rounds are queued without waiting: the host reads the round
// counters back once after the expected number of rounds (and once per
// further round in the rare case that more are needed).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "internal.hpp"

using namespace hss;

namespace hss {

hipError_t dev_alloc(MemSource* m, void** p, size_t bytes) {
    return m ? m->dev_get(p, bytes) : hipMalloc(p, bytes);
}

void dev_release(MemSource* m, void* p) {
    if (m) m->dev_put(p);
    else (void)hipFree(p);
}

hipError_t host_alloc(MemSource* m, void** p, size_t bytes) {
    return m ? m->host_get(p, bytes) : hipHostMalloc(p, bytes, hipHostMallocDefault);
}

void host_release(MemSource* m, void* p) {
    if (m) m->host_put(p);
    else (void)hipHostFree(p);
}

}  // namespace hss

namespace {

thread_local std::string g_last_error;

hss_status fail(hss_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? HSS_ERR_OUT_OF_MEMORY : HSS_ERR_DEVICE, \
                        std::string(#expr) + ": " + hipGetErrorString(e_));              \
    } while (0)

typedef unsigned __int128 u128;

constexpr uint32_t kMaxRestarts = 8;     // capacity growths per call
constexpr uint32_t kMaxRateRounds = 64;  // rounds kept in the rate table
// Expected first-round probes above which they are sorted by the segmented
// sort rather than ranked pairwise inside their interval.
constexpr uint64_t kBigRound = 16384;
constexpr uint64_t kPresampleMin = 1ull << 20;   // keys of a plan whose first draws go ahead
// Draws are taken ahead only for sparse samples (at most this many expected
// per round): the list costs a contended append per wave, and dense samples
// (one-round HSS, full samples) are better drawn by the per-slice sampler.
constexpr uint64_t kPresampleExpectMax = 1ull << 16;
// First round whose ranks are searched inside the probes' interval slices
// (round 1 has one interval, the whole input: searched by segment chunks).
constexpr uint32_t kPairRankFrom = 2;
constexpr uint32_t kDefaultSmallCap = 2048;
constexpr uint32_t kDefaultSampleGrid = 1024;
constexpr uint32_t kDefaultPairFrom = kPairRankFrom;
constexpr uint32_t kDefaultPairGrid = 8192;

struct RoundRecord {
    uint64_t domain = 0, m = 0;
    uint32_t thresh = 0, all = 0;
    std::vector<uint64_t> key, tag, rank;
    std::vector<uint64_t> lo, hi, chi;
    std::vector<uint8_t> settled;
    std::vector<uint32_t> counts;   // trace level 2: c_s(e) at [e p + s]
};

// Sub-allocation of one device arena.
struct Arena {
    char* base = nullptr;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T* p = (T*)(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
};

// Host view of one instance.
struct InstHost {
    uint64_t n = 0;
    uint32_t p = 0;       // segments
    uint32_t q = 0;       // buckets: p, or fewer in a stage of section 5.3
    double eps = 0;
    uint64_t tol = 0;     // section 2: the target range is N i/q +- tol
    uint32_t k = 1;       // rounds of the rate schedule (section 4.2)
    double a = 0;         // s_k = 2 ln q / eps
    uint64_t pos0 = 0, tab0 = 0;
    uint32_t seg0 = 0, row0 = 0;
    uint64_t max_seg = 0, max_bucket = 0;
};

// Every formula that counts buckets takes q (the splitters are i = 1..q-1):
// with q = p these are the constants of sections 2 and 4.2.
void instance_constants(InstHost& h, const hss_tuning& t) {
    const double nd = (double)h.n, qd = (double)h.q;
    h.tol = (uint64_t)std::floor((nd * h.eps) / (2.0 * qd));
    h.a = (2.0 * std::log(qd)) / h.eps;
    const double kk = std::ceil(std::log(h.a));
    h.k = (kk >= 1.0) ? (uint32_t)kk : 1u;
    if (t.k_override) h.k = t.k_override;
    h.max_seg = (h.n + h.p - 1) / h.p;
    h.max_bucket = (h.n + h.q - 1) / h.q + 2 * h.tol;
}

// Acceptance rule of round j: rate q_j = q s_j / N with s_j = a^(j/k),
// clamped at 1 ("take all").
// With a probe budget only round 1 is known here (its domain is all N keys);
// the device sets the later rounds from their measured domains.
void round_rate(const InstHost& h, const hss_tuning& t, uint32_t j, bool forced, uint32_t* thresh,
                int* all) {
    const double s_j = std::pow(h.a, (double)j / (double)h.k);
    const double q = t.probes_per_round
                         ? ((double)t.probes_per_round * (double)h.q) / (double)h.n
                         : ((double)h.q * s_j) / (double)h.n;
    if (q >= 1.0 || (forced && j == 1 && t.force_full_sample)) {
        *thresh = 0xFFFFFFFFu;
        *all = 1;
    } else {
        *thresh = (uint32_t)std::floor(q * 4294967296.0);
        *all = 0;
    }
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

// ------------------------------------------------------------- engine ----
struct Engine {
    int key_bytes = 8;
    bool payload = false;
    hss_tuning tune{};
    int device = 0;
    std::vector<InstHost> ih;
    uint64_t n_tot = 0;
    uint32_t S = 0, Q = 0;    // segments, splitter rows
    uint64_t T = 0;           // entries of the (q+1) x p tables
    uint32_t p_max = 0, J = 1, k_max = 1;
    uint64_t min_seg = 0;              // shortest segment the local sort's first level takes
    uint64_t max_seg = 0, max_bucket = 0;
    // engines of a batch read their inputs through per-segment source
    // addresses; segments above kDirectSegMax take the MSD pass from a list,
    // the others are sorted whole
    bool batch = false;
    bool listed = false;
    uint32_t n_msd = 0, msd_tiles = 0, n_direct = 0, n_chunks = 0;
    uint64_t n_fences = 0;

    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* B = nullptr;  uint64_t* Bv = nullptr;
    void* A = nullptr;  uint64_t* Av = nullptr;
    uint64_t* seg_off = nullptr;
    uint32_t* seg_inst = nullptr;
    uint32_t* row_inst = nullptr;
    uint64_t* ideal = nullptr;
    InstDesc* inst_d = nullptr;
    InstRun* run_d = nullptr;
    uint32_t* thresh_d = nullptr;
    uint8_t* all_d = nullptr;
    uint32_t* counts = nullptr;
    RoundArgs ra{};
    uint64_t* chi_all = nullptr;
    uint32_t* pick_bits = nullptr;
    uint32_t* dst = nullptr;
    uint32_t* chunk0 = nullptr;
    Fences fences;
    uint64_t* fence_base = nullptr;
    uint32_t* chunk_seg = nullptr;
    uint32_t* chunk_lo = nullptr;
    uint8_t* bucket_shift = nullptr;
    uint64_t* bucket_base = nullptr;
    uint64_t* sb_start = nullptr;
    uint32_t* sb_len = nullptr;
    OversizeList ov, ov2;
    EqualList eq;
    LevelWork lw;
    PackedJobs pj;
    SlowList sl;
    HybridHost hh;
    uint32_t* msd_seg = nullptr;
    uint64_t* msd_beg = nullptr;
    uint64_t* msd_end = nullptr;
    uint32_t* msd_tile_seg = nullptr;
    uint32_t* msd_tile0 = nullptr;
    uint32_t* direct_seg = nullptr;
    uint64_t* msd_src = nullptr;
    uint64_t* msd_vsrc = nullptr;
    uint64_t* direct_src = nullptr;
    uint64_t* direct_vsrc = nullptr;
    // key range of every MSD list entry (listed engines): the first local
    // sort takes its digit over it when first_shift is set
    uint8_t* msd_shift = nullptr;
    uint64_t* msd_base = nullptr;
    const uint8_t* first_shift = nullptr;
    const uint64_t* first_base = nullptr;
    // when set, the splitter ranks (Q words) are copied here once the rounds
    // end, and chi_ready is recorded after the copy (before the exchange)
    uint64_t* chi_out_host = nullptr;
    hipEvent_t chi_ready = nullptr;
    // one large instance: the draws of the first rounds are taken on a side
    // stream while the memory-bound local sort runs (they depend on the
    // seed and the tags only)
    uint32_t pre_rounds = 0;
    // rounds queued ahead of the exchange, not yet read back (0: none)
    uint32_t ahead_rounds = 0;
    uint32_t pre_thresh[kPreRounds] = {};
    uint32_t pre_cap = 0;
    uint32_t* pre_mem = nullptr;        // kPreRounds counts, then pre_rounds lists of pre_cap tags
    hipStream_t aux = nullptr;
    hipEvent_t ev_start = nullptr, ev_pre = nullptr;
    uint64_t cur_seed = 0;              // seed of the call in progress
    bool sort_counted = false;          // the bucket sort's first counts came with the exchange

    uint64_t counts_words = 0;

    // round 1 of a plan whose first sample is large (one-round HSS, a full
    // sample): its probes are sorted by the segmented sort, in scratch
    // grown on demand
    bool big_first = false;
    void* psort_mem = nullptr;
    uint64_t psort_cap = 0;

    // probes and count matrix, grown on demand
    void* probe_mem = nullptr;
    size_t probe_bytes = 0;
    uint64_t cap = 0;
    uint32_t* cmat = nullptr;
    uint64_t cm_cap = 0;

    RoundCounters* h_ctr = nullptr;   // pinned; 32 more bytes for the sort's read-back
    InstRun* h_run = nullptr;         // pinned
    RoundHist* h_hist = nullptr;      // pinned, J entries
    std::vector<RoundRecord> trace;
    Profiler prof;

    // where the memory comes from (null: hipMalloc), and the one stream a
    // server engine runs on (null: plans and batches, any stream)
    MemSource* mem = nullptr;
    hipStream_t own_stream = nullptr;
    // the workspace is one fixed region (the static scratch array): no side
    // stream, no captured graph, probe buffers sized once with headroom
    bool fixed_mem = false;

    // the first rounds of a call as a captured graph, for the probe and
    // count-matrix buffers and the knobs it was captured with
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t rounds_exec = nullptr;
    uint32_t rounds_exec_n = 0;
    uint64_t rounds_exec_cap = 0, rounds_exec_cm = 0;
    uint32_t rounds_exec_knobs = 0;

    // launch knobs (none changes an output); knob_gen counts changes
    hss_knobs knobs{kDefaultSmallCap, kDefaultSampleGrid, kDefaultPairFrom, kDefaultPairGrid, 0};
    uint32_t knob_gen = 0;

    ~Engine() {
        if (!arena && !probe_mem && !aux) return;   // never set up on a device
        (void)hipSetDevice(device);
        if (own_stream) (void)hipStreamSynchronize(own_stream);
        else (void)hipDeviceSynchronize();
        if (rounds_exec) (void)hipGraphExecDestroy(rounds_exec);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
        if (ev_start) (void)hipEventDestroy(ev_start);
        if (ev_pre) (void)hipEventDestroy(ev_pre);
        if (hh.flag_ev) (void)hipEventDestroy(hh.flag_ev);
        if (pre_mem) dev_release(mem, pre_mem);
        for (void* q : {probe_mem, psort_mem, (void*)cmat, (void*)hh.fb_counts, (void*)hh.fb_sb_start,
                        (void*)hh.fb_sb_len, arena})
            if (q) dev_release(mem, q);
        for (void* q : {(void*)h_ctr, (void*)h_run, (void*)h_hist})
            if (q) host_release(mem, q);
    }
};

struct hss_plan_s {
    Engine e;
};

struct hss_batch_s {
    Engine* eng[2] = {nullptr, nullptr};   // u32 instances, u64 instances
    std::vector<std::pair<int, uint32_t>> where;   // instance -> (engine, index in it)
    // with both key widths present, the u64 engine runs on a stream of its own
    // (from a second host thread) beside the u32 engine on the caller's stream
    hipStream_t side = nullptr;
    hipEvent_t ev_in = nullptr;
    ~hss_batch_s() {
        delete eng[0];
        delete eng[1];
        if (side) (void)hipStreamDestroy(side);
        if (ev_in) (void)hipEventDestroy(ev_in);
    }
};

namespace {

// Host tables of the instance layout (positions, segments, rows, lists).
struct Layout {
    std::vector<uint64_t> seg_off, ideal, fence_base, msd_beg, msd_end;
    std::vector<uint32_t> seg_inst, row_inst, chunk_seg, chunk_lo, msd_seg, msd_tile_seg, msd_tile0,
        direct_seg, thresh;
    std::vector<uint8_t> all;
    std::vector<InstDesc> inst;
};

void build_layout(Engine& E, Layout& L) {
    const uint32_t B = (uint32_t)E.ih.size();
    uint64_t pos = 0, tab = 0;
    uint32_t seg = 0, row = 0;
    E.p_max = 0;
    E.k_max = 1;
    E.max_seg = 0;
    E.max_bucket = 0;
    E.min_seg = ~0ull;
    for (InstHost& h : E.ih) {
        h.pos0 = pos;
        h.seg0 = seg;
        h.row0 = row;
        h.tab0 = tab;
        pos += h.n;
        seg += h.p;
        row += h.q + 1;
        tab += (uint64_t)(h.q + 1) * h.p;
        E.p_max = std::max(E.p_max, h.p);
        E.k_max = std::max(E.k_max, h.k);
        E.max_seg = std::max(E.max_seg, h.max_seg);
        E.min_seg = std::min(E.min_seg, h.n / h.p);   // segments of floor(n / p) keys or one more
        E.max_bucket = std::max(E.max_bucket, h.max_bucket);
    }
    E.n_tot = pos;
    E.S = seg;
    E.Q = row;
    E.T = tab;
    E.listed = E.batch;
    L.seg_off.assign(E.S + 1, 0);
    L.seg_inst.assign(E.S, 0);
    L.row_inst.assign(E.Q, 0);
    L.ideal.assign(E.Q, 0);
    L.inst.assign(B, InstDesc{});
    for (uint32_t I = 0; I < B; ++I) {
        const InstHost& h = E.ih[I];
        // segment boundaries floor(s N / p) and ideal ranks floor(i N / q)
        // (section 2; the same integers when q = p)
        for (uint32_t s = 0; s < h.p; ++s) {
            L.seg_off[h.seg0 + s] = h.pos0 + (uint64_t)(((u128)s * h.n) / h.p);
            L.seg_inst[h.seg0 + s] = I;
        }
        for (uint32_t i = 0; i <= h.q; ++i) {
            L.row_inst[h.row0 + i] = I;
            L.ideal[h.row0 + i] = (uint64_t)(((u128)i * h.n) / h.q);
        }
        InstDesc& d = L.inst[I];
        d.n = h.n;
        d.pos0 = h.pos0;
        d.tol = h.tol;
        d.tab0 = h.tab0;
        d.p = h.p;
        d.seg0 = h.seg0;
        d.row0 = h.row0;
        d.q = h.q;
    }
    L.seg_off[E.S] = E.n_tot;
    // fences and rank chunks of every segment
    L.fence_base.assign(E.S + 1, 0);
    L.chunk_seg.clear();
    L.chunk_lo.clear();
    for (uint32_t s = 0; s < E.S; ++s) {
        const uint64_t len = L.seg_off[s + 1] - L.seg_off[s];
        L.fence_base[s + 1] = L.fence_base[s] + (len + kFenceStride - 1) / kFenceStride;
        for (uint64_t lo = 0; lo < len; lo += kRankChunk) {
            L.chunk_seg.push_back(s);
            L.chunk_lo.push_back((uint32_t)lo);
        }
    }
    E.n_fences = L.fence_base[E.S];
    E.n_chunks = (uint32_t)L.chunk_seg.size();
    // segment lists of the local sort
    E.n_msd = E.n_direct = E.msd_tiles = 0;
    L.msd_seg.clear();
    L.msd_beg.clear();
    L.msd_end.clear();
    L.msd_tile_seg.clear();
    L.msd_tile0.assign(1, 0);
    L.direct_seg.clear();
    if (E.listed) {
        for (uint32_t s = 0; s < E.S; ++s) {
            const uint64_t len = L.seg_off[s + 1] - L.seg_off[s];
            if (len <= kDirectSegMax) {
                L.direct_seg.push_back(s);
                continue;
            }
            if (L.msd_seg.empty()) E.min_seg = len;
            E.min_seg = std::min(E.min_seg, len);
            const uint32_t li = (uint32_t)L.msd_seg.size();
            L.msd_seg.push_back(s);
            L.msd_beg.push_back(L.seg_off[s]);
            L.msd_end.push_back(L.seg_off[s + 1]);
            const uint32_t nt = (uint32_t)((len + kSortTile - 1) / kSortTile);
            for (uint32_t t = 0; t < nt; ++t) L.msd_tile_seg.push_back(li);
            L.msd_tile0.push_back(L.msd_tile0.back() + nt);
        }
        E.n_msd = (uint32_t)L.msd_seg.size();
        E.n_direct = (uint32_t)L.direct_seg.size();
        E.msd_tiles = L.msd_tile0.back();
    }
    // rate table: rounds until every instance takes all keys of its domain
    E.J = 1;
    for (const InstHost& h : E.ih) {
        uint32_t j = 1;
        for (; j < kMaxRateRounds; ++j) {
            uint32_t t;
            int al;
            round_rate(h, E.tune, j, true, &t, &al);
            if (al) break;
        }
        // a probe budget has no schedule: any number of rounds up to the cap
        E.J = std::max(E.J, E.tune.probes_per_round ? kMaxRateRounds : j);
    }
    L.thresh.assign((size_t)B * E.J, 0);
    L.all.assign((size_t)B * E.J, 0);
    for (uint32_t I = 0; I < B; ++I)
        for (uint32_t j = 1; j <= E.J; ++j) {
            uint32_t t;
            int al;
            round_rate(E.ih[I], E.tune, j, true, &t, &al);
            L.thresh[(size_t)I * E.J + j - 1] = t;
            L.all[(size_t)I * E.J + j - 1] = (uint8_t)al;
        }
    // the first round samples every key at the first rate: its expected
    // probe count decides how its probes are put in order
    if (B == 1 && E.J >= 1) {
        const double m1 = L.all[0] ? (double)E.ih[0].n : (double)E.ih[0].n * (double)L.thresh[0] / 4294967296.0;
        E.big_first = m1 > (double)kBigRound;
    }
}

uint64_t tiles_of(uint64_t len) { return (len + kSortTile - 1) / kSortTile; }


size_t layout(Engine& E, char* base) {
    Arena ar;
    ar.base = base;
    const uint64_t n = E.n_tot;
    const uint32_t S = E.S, Q = E.Q, B = (uint32_t)E.ih.size();
    E.B = ar.take<char>(n * E.key_bytes);
    E.A = ar.take<char>(n * E.key_bytes);
    E.Bv = E.payload ? ar.take<uint64_t>(n) : nullptr;
    E.Av = E.payload ? ar.take<uint64_t>(n) : nullptr;
    E.seg_off = ar.take<uint64_t>(S + 1);
    E.seg_inst = ar.take<uint32_t>(S);
    E.row_inst = ar.take<uint32_t>(Q);
    E.ideal = ar.take<uint64_t>(Q);
    E.inst_d = ar.take<InstDesc>(B);
    E.run_d = ar.take<InstRun>(B);
    E.thresh_d = ar.take<uint32_t>((size_t)B * E.J);
    E.all_d = ar.take<uint8_t>((size_t)B * E.J);
    // count table: the MSD pass of the local sort, and of the bucket sort
    // (one instance only)
    uint64_t tiles = E.listed ? E.msd_tiles : (uint64_t)S * tiles_of(E.max_seg);
    if (!E.listed) tiles = std::max(tiles, (uint64_t)E.ih[0].q * tiles_of(E.max_bucket));
    E.counts = ar.take<uint32_t>(tiles * 256 + 256);
    E.counts_words = tiles * 256 + 256;
    RoundArgs& r = E.ra;
    r.settled = ar.take<uint32_t>(Q);
    r.chi = ar.take<uint64_t>(Q);
    r.lrank = ar.take<uint64_t>(Q);
    r.urank = ar.take<uint64_t>(Q);
    r.s_key = ar.take<uint64_t>(Q);
    r.s_tag = ar.take<uint64_t>(Q);
    r.l_tag = ar.take<uint64_t>(Q);
    r.u_tag = ar.take<uint64_t>(Q);
    r.lpos = ar.take<uint32_t>(E.T);
    r.upos = ar.take<uint32_t>(E.T);
    r.prow = ar.take<uint32_t>(E.T);
    r.ivl_row = ar.take<uint32_t>(Q);
    r.ivl_inst = ar.take<uint32_t>(Q);
    r.ivl_tot = ar.take<uint64_t>(Q + 1);
    r.ivl_nz = ar.take<uint32_t>(Q + 1);
    r.ivl_dom = ar.take<uint64_t>(Q + 1);
    r.ivl_pcnt = ar.take<uint32_t>(Q);
    r.ivl_poff = ar.take<uint32_t>(Q + 1);
    r.ivl_cursor = ar.take<uint32_t>(Q);
    r.ivl_tile0 = ar.take<uint32_t>(Q + 1);
    r.ivl_lkey = ar.take<uint64_t>(Q);
    r.ivl_ltag = ar.take<int64_t>(Q);
    r.ivl_ukey = ar.take<uint64_t>(Q);
    r.ivl_utag = ar.take<int64_t>(Q);
    r.slices = ar.take<uint4>(E.T > 0 ? E.T : 1);
    r.inst_plo = ar.take<uint32_t>(B);
    r.inst_pm = ar.take<uint32_t>(B);
    r.cm_off = ar.take<uint64_t>(B);
    r.sel_e = ar.take<uint32_t>(2 * (size_t)Q);
    r.sel_kind = ar.take<uint8_t>(2 * (size_t)Q);
    r.ctr = ar.take<RoundCounters>(1);
    r.hist = ar.take<RoundHist>(E.J);
    E.chi_all = ar.take<uint64_t>(Q);
    // section 6's sampler: one bit per tag (each instance starts at a word)
    E.pick_bits = E.tune.pick_sampler ? ar.take<uint32_t>(n / 32 + 2 * (size_t)B + 1) : nullptr;
    E.dst = ar.take<uint32_t>(E.T > 0 ? E.T : 1);
    E.chunk0 = ar.take<uint32_t>(Q + 1);
    E.fence_base = ar.take<uint64_t>(S + 1);
    E.fences.key = ar.take<uint64_t>(E.n_fences + 1);
    E.chunk_seg = ar.take<uint32_t>(E.n_chunks + 1);
    E.chunk_lo = ar.take<uint32_t>(E.n_chunks + 1);
    E.bucket_shift = ar.take<uint8_t>(S);
    E.bucket_base = ar.take<uint64_t>(S);
    const uint32_t msd_segs = E.listed ? E.n_msd : S;
    E.sb_start = ar.take<uint64_t>((size_t)msd_segs * 256 + 1);
    E.sb_len = ar.take<uint32_t>((size_t)msd_segs * 256 + 1);
    // the lists of the hybrid sort (capacities from the key count alone)
    const uint64_t ovc = oversize_capacity(n);
    uint32_t* list_err = ar.take<uint32_t>(1);
    for (OversizeList* o : {&E.ov, &E.ov2}) {
        o->count = ar.take<uint32_t>(1);
        o->tiles = ar.take<uint32_t>(1);
        o->summary = ar.take<uint32_t>(8);
        o->beg = ar.take<uint64_t>(ovc);
        o->end = ar.take<uint64_t>(ovc);
        o->base = ar.take<uint64_t>(ovc);
        o->seg = ar.take<uint32_t>(ovc);
        o->bits = ar.take<uint8_t>(ovc);
        o->loc = ar.take<uint8_t>(ovc);
        o->src = ar.take<uint64_t>(ovc);
        o->vsrc = ar.take<uint64_t>(ovc);
        o->tile0 = ar.take<uint32_t>(ovc + 1);
        o->tile_seg = ar.take<uint32_t>(oversize_tile_capacity(n));
        o->capacity = (uint32_t)ovc;
        o->err = list_err;
    }
    E.eq.count = ar.take<uint32_t>(1);
    E.eq.beg = ar.take<uint64_t>(ovc);
    E.eq.end = ar.take<uint64_t>(ovc);
    E.eq.seg = ar.take<uint32_t>(ovc);
    E.eq.loc = ar.take<uint8_t>(ovc);
    E.eq.src = ar.take<uint64_t>(ovc);
    E.eq.vsrc = ar.take<uint64_t>(ovc);
    E.eq.capacity = (uint32_t)ovc;
    E.eq.err = list_err;
    const uint64_t lwc = level_capacity(msd_segs, n);
    E.lw.shift = ar.take<uint8_t>(lwc);
    E.lw.skip = ar.take<uint8_t>(lwc);
    E.lw.dst = ar.take<uint64_t>(lwc);
    E.lw.vdst = ar.take<uint64_t>(lwc);
    E.lw.and_mask = ar.take<uint64_t>(lwc);
    E.lw.or_mask = ar.take<uint64_t>(lwc);
    // splitter tables of a level's entries
    E.lw.splits = ar.take<uint64_t>(lwc * kSplitSlots);
    E.lw.n_splits = ar.take<uint32_t>(lwc);
    E.lw.split_entries = ar.take<uint32_t>(1);
    const uint64_t pjc = packed_capacity(n);
    E.pj.count = ar.take<uint32_t>(1);
    E.pj.start = ar.take<uint64_t>(pjc);
    E.pj.len = ar.take<uint32_t>(pjc);
    E.pj.entry = ar.take<uint32_t>(pjc);
    E.pj.base = ar.take<uint64_t>(pjc);
    E.pj.bits = ar.take<uint8_t>(pjc);
    E.pj.capacity = (uint32_t)pjc;
    E.pj.err = list_err;
    const uint64_t stc = stage_capacity(msd_segs, n);
    E.pj.s_start = ar.take<uint64_t>(stc);
    E.pj.s_len = ar.take<uint32_t>(stc);
    E.pj.s_base = ar.take<uint64_t>(stc);
    E.pj.s_bits = ar.take<uint8_t>(stc);
    E.pj.s_capacity = stc;
    E.pj.n_of = ar.take<uint32_t>(lwc + 1);
    E.pj.chunk_sum = ar.take<uint32_t>(lwc / kPackChunk + 2);
    const uint64_t slc = slow_capacity(n);
    E.sl.count = ar.take<uint32_t>(1);
    E.sl.beg = ar.take<uint64_t>(slc);
    E.sl.len = ar.take<uint32_t>(slc);
    E.sl.seg = ar.take<uint32_t>(slc);
    E.sl.capacity = (uint32_t)slc;
    E.sl.err = list_err;
    if (E.listed) {
        E.msd_seg = ar.take<uint32_t>(E.n_msd + 1);
        E.msd_beg = ar.take<uint64_t>(E.n_msd + 1);
        E.msd_end = ar.take<uint64_t>(E.n_msd + 1);
        E.msd_tile_seg = ar.take<uint32_t>(E.msd_tiles + 1);
        E.msd_tile0 = ar.take<uint32_t>(E.n_msd + 1);
        E.direct_seg = ar.take<uint32_t>(E.n_direct + 1);
        E.msd_src = ar.take<uint64_t>(E.n_msd + 1);
        E.msd_vsrc = ar.take<uint64_t>(E.n_msd + 1);
        E.msd_shift = ar.take<uint8_t>(E.n_msd + 1);
        E.msd_base = ar.take<uint64_t>(E.n_msd + 1);
        E.direct_src = ar.take<uint64_t>(E.n_direct + 1);
        E.direct_vsrc = ar.take<uint64_t>(E.n_direct + 1);
    }
    return ar.used;
}

// The probe arrays for `cap` probes laid out from `ar` (a null base only
// measures); returns the bytes taken.
size_t probe_layout(RoundArgs& r, Arena& ar, uint64_t cap) {
    r.pr_key = ar.take<uint64_t>(cap);
    r.pr_tag = ar.take<uint64_t>(cap);
    r.pr_ivl = ar.take<uint32_t>(cap);
    r.g_key = ar.take<uint64_t>(cap);
    r.g_tag = ar.take<uint64_t>(cap);
    r.ps_key = ar.take<uint64_t>(cap);
    r.ps_tag = ar.take<uint64_t>(cap);
    r.ps_ivl = ar.take<uint32_t>(cap);
    r.ps_seg = ar.take<uint32_t>(cap);
    r.ps_row = ar.take<uint32_t>(cap);
    r.pr_rank = ar.take<uint64_t>(cap);
    return ar.used + 256;
}

size_t probe_bytes_for(uint64_t cap) {
    RoundArgs tmp{};
    Arena ar;
    return probe_layout(tmp, ar, cap);
}

// Probe buffers for `need` probes and a count matrix of `cm_need` words.
hss_status grow(Engine& E, uint64_t need, uint64_t cm_need) {
    RoundArgs& r = E.ra;
    if (E.tune.workspace_limit_mib) {
        // the probe buffers and count matrix this growth would leave
        uint64_t cap = E.cap ? E.cap : 4096, words = E.cm_cap ? E.cm_cap : (1ull << 20);
        while (cap < need) cap *= 2;
        while (words < cm_need) words *= 2;
        const uint64_t total = E.arena_bytes + probe_bytes_for(cap) + words * 4;
        if (total > ((uint64_t)E.tune.workspace_limit_mib << 20))
            return fail(HSS_ERR_OUT_OF_MEMORY, "probe buffers of " + std::to_string(cap) +
                                                   " probes would exceed the workspace limit");
    }
    if (need > E.cap || !E.probe_mem) {
        uint64_t cap = E.cap ? E.cap : 4096;
        while (cap < need) cap *= 2;
        if (E.probe_mem) dev_release(E.mem, E.probe_mem);
        E.probe_mem = nullptr;
        E.cap = 0;
        E.probe_bytes = probe_bytes_for(cap);
        HIP_TRY(dev_alloc(E.mem, &E.probe_mem, E.probe_bytes));
        Arena ar;
        ar.base = (char*)E.probe_mem;
        probe_layout(r, ar, cap);
        E.cap = cap;
        r.cap = cap;
    }
    if (cm_need > E.cm_cap || !E.cmat) {
        uint64_t want = E.cm_cap ? E.cm_cap : (1ull << 20);
        while (want < cm_need) want *= 2;
        if (E.cmat) dev_release(E.mem, E.cmat);
        E.cmat = nullptr;
        E.cm_cap = 0;
        HIP_TRY(dev_alloc(E.mem, (void**)&E.cmat, want * 4));
        E.cm_cap = want;
        r.cmat = E.cmat;
        r.cm_cap = want;
    }
    return HSS_OK;
}

// Host tables to the device: synchronously, or on the engine's own stream
// (the vectors outlive the copies: the caller synchronises that stream).
template <typename T>
hipError_t h2d(T* d, const std::vector<T>& v, hipStream_t s = nullptr) {
    if (v.empty()) return hipSuccess;
    if (s) return hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Initial probe capacity and count-matrix words: a generous multiple of the
// expected sample q s_j / s_{j-1} per round and instance (more headroom in a
// fixed region, which cannot grow); the count matrix holds each instance's
// probes x p.
void probe_sizes(const Engine& E, uint64_t* want, uint64_t* cm) {
    *want = 0;
    *cm = 0;
    for (const InstHost& h : E.ih) {
        const uint64_t m = E.fixed_mem ? std::min<uint64_t>(h.n, 32ull * h.q + 4096)
                                       : std::min<uint64_t>(h.n, 8ull * h.q + 256);
        *want += m;
        *cm += m * h.p;
    }
}

// Device bytes of an engine's workspace at set-up: its arena (layout), the
// first probe buffers and count matrix (grown on demand, never shrunk), and,
// in a fixed region, the deeper levels' count tables at their bounds.
uint64_t workspace_estimate(Engine& E) {
    auto up = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
    uint64_t b = up(layout(E, nullptr) + 256);
    uint64_t want = 0, cm = 0;
    probe_sizes(E, &want, &cm);
    uint64_t cap = 4096;
    while (cap < want) cap *= 2;
    b += up(probe_bytes_for(cap));
    uint64_t words = 1ull << 20;
    while (words < cm) words *= 2;
    b += up(words * 4);
    if (E.fixed_mem) {
        const uint64_t fbw = oversize_tile_capacity(E.n_tot) * 256, fbs = oversize_capacity(E.n_tot) * 256 + 1;
        b += up(fbw * 4) + up(fbs * 8) + up(fbs * 4);
    }
    return b;
}

// Allocates the engine for its instances (E.ih filled, constants computed).
hss_status engine_init(Engine& E) {
    Layout L;
    build_layout(E, L);
    if (E.n_tot >= (1ull << 32)) return fail(HSS_ERR_UNSUPPORTED, "more than 2^32 - 1 keys in one plan");
    if (E.max_bucket >= (1ull << 32)) return fail(HSS_ERR_UNSUPPORTED, "bucket bound >= 2^32");
    E.arena_bytes = layout(E, nullptr) + 256;
    // the workspace limit is checked on the host, before any device call
    if (E.tune.workspace_limit_mib) {
        const uint64_t need = workspace_estimate(E);
        const uint64_t limit = (uint64_t)E.tune.workspace_limit_mib << 20;
        if (need > limit)
            return fail(HSS_ERR_OUT_OF_MEMORY, "the workspace needs " + std::to_string(need) +
                                                   " bytes, above the limit of " + std::to_string(limit));
    }
    HIP_TRY(hipGetDevice(&E.device));
    E.hh.mem = E.mem;
    HIP_TRY(dev_alloc(E.mem, &E.arena, E.arena_bytes));
    layout(E, (char*)E.arena);
    HIP_TRY(host_alloc(E.mem, (void**)&E.h_ctr, sizeof(RoundCounters) + 32));
    E.hh.pinned = (uint32_t*)((char*)E.h_ctr + sizeof(RoundCounters));
    if (!E.fixed_mem) HIP_TRY(hipEventCreateWithFlags(&E.hh.flag_ev, hipEventDisableTiming));
    HIP_TRY(host_alloc(E.mem, (void**)&E.h_run, E.ih.size() * sizeof(InstRun)));
    HIP_TRY(host_alloc(E.mem, (void**)&E.h_hist, E.J * sizeof(RoundHist)));
    hipStream_t cs = E.own_stream;
    HIP_TRY(h2d(E.seg_off, L.seg_off, cs));
    HIP_TRY(h2d(E.seg_inst, L.seg_inst, cs));
    HIP_TRY(h2d(E.row_inst, L.row_inst, cs));
    HIP_TRY(h2d(E.ideal, L.ideal, cs));
    HIP_TRY(h2d(E.inst_d, L.inst, cs));
    HIP_TRY(h2d(E.thresh_d, L.thresh, cs));
    HIP_TRY(h2d(E.all_d, L.all, cs));
    HIP_TRY(h2d(E.fence_base, L.fence_base, cs));
    HIP_TRY(h2d(E.chunk_seg, L.chunk_seg, cs));
    HIP_TRY(h2d(E.chunk_lo, L.chunk_lo, cs));
    if (E.listed) {
        HIP_TRY(h2d(E.msd_seg, L.msd_seg, cs));
        HIP_TRY(h2d(E.msd_beg, L.msd_beg, cs));
        HIP_TRY(h2d(E.msd_end, L.msd_end, cs));
        HIP_TRY(h2d(E.msd_tile_seg, L.msd_tile_seg, cs));
        HIP_TRY(h2d(E.msd_tile0, L.msd_tile0, cs));
        HIP_TRY(h2d(E.direct_seg, L.direct_seg, cs));
    }
    if (cs) HIP_TRY(hipStreamSynchronize(cs));   // L goes out of scope
    E.fences.base = E.fence_base;
    E.fences.seg_off = E.seg_off;
    RoundArgs& r = E.ra;
    r.key_bytes = E.key_bytes;
    r.B = E.B;
    r.n_inst = (uint32_t)E.ih.size();
    r.n_rows = E.Q;
    r.n_segs = E.S;
    r.p_max = E.p_max;
    r.J = E.J;
    r.inst = E.inst_d;
    r.run = E.run_d;
    r.thresh = E.thresh_d;
    r.all = E.all_d;
    r.budget = E.tune.probes_per_round;
    r.picks = E.tune.pick_sampler ? 1u : 0u;
    r.pick_bits = E.pick_bits;
    r.pick_words = E.pick_bits ? E.n_tot / 32 + 2 * E.ih.size() + 1 : 0;
    r.pair_rank_from = E.knobs.pair_rank_from;
    r.sample_grid = E.knobs.sample_workgroups;
    r.pair_grid = E.knobs.pair_rank_workgroups;
    r.dense_rank = 0;
    r.seg_off = E.seg_off;
    r.seg_inst = E.seg_inst;
    r.row_inst = E.row_inst;
    r.ideal = E.ideal;
    r.chunk_seg = E.chunk_seg;
    r.chunk_lo = E.chunk_lo;
    r.n_chunks = E.n_chunks;
    r.fences = E.fences;
    // draws taken ahead: the first rounds (up to kPreRounds) of one instance
    // of at least kPresampleMin keys, while their rate is fixed and below 1
    // (with a probe budget only round 1's is)
    for (uint32_t j = 0; j < kPreRounds; ++j) {
        r.pre_list[j] = nullptr;
        r.pre_cnt[j] = nullptr;
    }
    r.pre_cap = 0;
    E.pre_rounds = 0;
    double expect = 0;   // largest expected number of draws below a threshold
    if (!E.batch && !E.fixed_mem && !E.own_stream && E.ih.size() == 1 && E.n_tot >= kPresampleMin &&
        !E.tune.lsd_only && !E.tune.pick_sampler) {
        for (uint32_t j = 1; j <= kPreRounds && j <= E.J; ++j) {
            if (L.all[j - 1] || (j > 1 && E.tune.probes_per_round)) break;
            // rounds whose lists would be long draw by themselves
            const double e = (double)E.n_tot * ((double)L.thresh[j - 1] / 4294967296.0);
            if (e > (double)kPresampleExpectMax) break;
            E.pre_thresh[j - 1] = L.thresh[j - 1];
            expect = std::max(expect, e);
            E.pre_rounds = j;
        }
    }
    // a list of twice the expected draws plus 4096 holds all of them except
    // with negligible probability (binomial counts); a fuller one is not
    // used (the sampler draws itself)
    if (E.pre_rounds) {
        E.pre_cap = (uint32_t)(expect * 2 + 4096);
        HIP_TRY(dev_alloc(E.mem, (void**)&E.pre_mem,
                          (kPreRounds + (uint64_t)E.pre_cap * E.pre_rounds) * sizeof(uint32_t)));
        HIP_TRY(hipStreamCreateWithFlags(&E.aux, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&E.ev_start, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&E.ev_pre, hipEventDisableTiming));
        r.pre_cap = E.pre_cap;
        for (uint32_t j = 0; j < E.pre_rounds; ++j) {
            r.pre_cnt[j] = E.pre_mem + j;
            r.pre_list[j] = E.pre_mem + kPreRounds + (uint64_t)j * E.pre_cap;
        }
    }
    // probes: a generous multiple of the expected sample p s_j / s_{j-1} per
    // round and instance; the count matrix holds each instance's probes x p
    uint64_t want = 0, cm = 0;
    probe_sizes(E, &want, &cm);
    hss_status st = grow(E, want, cm);
    if (st != HSS_OK || !E.fixed_mem) return st;
    // a fixed region also holds the count tables of the deeper sort levels at
    // their bounds, so that no later call takes more of it
    const uint64_t fbw = oversize_tile_capacity(E.n_tot) * 256, fbs = oversize_capacity(E.n_tot) * 256 + 1;
    HIP_TRY(dev_alloc(E.mem, (void**)&E.hh.fb_counts, fbw * 4));
    HIP_TRY(dev_alloc(E.mem, (void**)&E.hh.fb_sb_start, fbs * 8));
    HIP_TRY(dev_alloc(E.mem, (void**)&E.hh.fb_sb_len, fbs * 4));
    E.hh.fb_words = fbw;
    E.hh.fb_sb = fbs;
    return HSS_OK;
}

hss_status read_counters(Engine& E, hipStream_t s, uint32_t rounds = 0) {
    HIP_TRY(hipMemcpyAsync(E.h_ctr, E.ra.ctr, sizeof(RoundCounters), hipMemcpyDeviceToHost, s));
    if (rounds)
        HIP_TRY(hipMemcpyAsync(E.h_hist, E.ra.hist, rounds * sizeof(RoundHist), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HSS_OK;
}

template <typename T>
hss_status d2h(std::vector<T>& v, const T* d, size_t count, hipStream_t s) {
    v.resize(count);
    if (count) HIP_TRY(hipMemcpyAsync(v.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    return HSS_OK;
}

// Local sort of every segment (first=true: of the callers' inputs) or of
// every bucket of the one instance (first=false).
hss_status segment_sort(Engine& E, bool first, const void* kin, const uint64_t* vin, void* kout,
                        uint64_t* vout, void* ktmp, uint64_t* vtmp, const uint64_t* seg_off,
                        uint32_t num_segs, uint64_t max_len, const uint8_t* seg_shift,
                        const uint64_t* seg_base, bool with_fences, hipStream_t s) {
    if (E.tune.lsd_only) {
        if (E.listed) return fail(HSS_ERR_UNSUPPORTED, "lsd_only in a batch");
        if (!kin || (E.payload && !vin)) return fail(HSS_ERR_INVALID_ARG, "segment sort without an input buffer");
        SegSort ss;
        ss.key_bytes = E.key_bytes;
        ss.keys_in = kin;
        ss.vals_in = vin;
        ss.keys_out = kout;
        ss.vals_out = vout;
        ss.keys_tmp = ktmp;
        ss.vals_tmp = vtmp;
        ss.seg_off = seg_off;
        ss.num_segs = num_segs;
        ss.max_seg_len = max_len;
        ss.total_len = E.n_tot;
        ss.counts = E.counts;
        ss.begin_bit = 0;
        ss.end_bit = E.key_bytes * 8;
        ss.prof = &E.prof;
        HIP_TRY(segmented_radix_sort(ss, s));
        if (with_fences) HIP_TRY(write_fences(kout, E.key_bytes, num_segs, E.fences, s));
        return HSS_OK;
    }
    // a batch reads its inputs through the segment sources; anything else
    // needs the input buffer itself
    if (!(first && E.listed) && (!kin || (E.payload && !vin)))
        return fail(HSS_ERR_INVALID_ARG, "segment sort without an input buffer");
    HybridSort hs;
    hs.key_bytes = E.key_bytes;
    hs.keys_in = kin;
    hs.vals_in = vin;
    hs.keys_out = kout;
    hs.vals_out = vout;
    hs.keys_tmp = ktmp;
    hs.vals_tmp = vtmp;
    hs.seg_off = seg_off;
    hs.num_segs = num_segs;
    hs.max_seg_len = max_len;
    hs.total_len = E.n_tot;
    hs.counts = E.counts;
    hs.sb_start = E.sb_start;
    hs.sb_len = E.sb_len;
    hs.seg_shift = seg_shift;
    hs.seg_base = seg_base;
    if (with_fences) hs.fences = E.fences;
    hs.ov = E.ov;
    hs.ov2 = E.ov2;
    hs.eq = E.eq;
    hs.lw = E.lw;
    hs.pj = E.pj;
    hs.sl = E.sl;
    hs.prof = &E.prof;
    hs.cap_large = first && E.knobs.small_sort_cap > 2048;
    hs.counted = !first && E.sort_counted;
    hs.min_seg_len = first ? E.min_seg : 0;
    if (first && E.listed) {
        hs.num_segs = E.n_msd;
        hs.msd_seg = E.msd_seg;
        hs.msd_beg = E.msd_beg;
        hs.msd_end = E.msd_end;
        hs.msd_tile_seg = E.msd_tile_seg;
        hs.msd_tile0 = E.msd_tile0;
        hs.msd_tiles = E.msd_tiles;
        hs.msd_src = E.msd_src;
        hs.msd_vsrc = E.payload ? E.msd_vsrc : nullptr;
        hs.direct_seg = E.direct_seg;
        hs.n_direct = E.n_direct;
        hs.direct_src = E.direct_src;
        hs.direct_vsrc = E.payload ? E.direct_vsrc : nullptr;
        hs.has_payload = E.payload;
    }
    HIP_TRY(hybrid_sort(hs, s, E.hh));
    return HSS_OK;
}

// Counts and rate of round j from its device history (read back).
void record_round(Engine& E, RoundRecord& rec, uint32_t j) {
    const RoundHist& h = E.h_hist[j - 1];
    rec.domain = h.domain;
    rec.m = h.m;
    rec.thresh = h.thresh;
    rec.all = h.all;
}

// The trace without tracing: counts of every round up to j that had
// unsettled splitters, from the history read back with the counters.
void record_history(Engine& E, uint32_t j) {
    for (uint32_t q = 0; q < j; ++q) {
        const RoundHist& h = E.h_hist[q];
        if (h.unsettled == 0) break;
        RoundRecord rec;
        record_round(E, rec, q + 1);
        E.trace.push_back(std::move(rec));
    }
}

// Round 1 of a plan whose first sample is large (one-round HSS, a full
// sample): the probes of its one interval are put in (key, tag) order by two
// stable segmented sorts, by tag and then by key, instead of the pairwise
// ranking inside the interval.
hss_status big_first_round(Engine& E, hipStream_t s) {
    RoundArgs& r = E.ra;
    HIP_TRY(launch_round_head(r, 1, s));
    hss_status st = read_counters(E, s, 0);
    if (st != HSS_OK) return st;
    const RoundCounters c = *E.h_ctr;
    const uint64_t m = c.m_stored;
    const uint32_t nivl = c.n_ivl;
    const uint32_t msd_segs = E.listed ? E.n_msd : E.S;
    const bool fits = !c.overflow && m > 0 && nivl >= 1 && m <= E.n_tot &&
                      (uint64_t)nivl * tiles_of(m) * 256 + 256 <= E.counts_words &&
                      nivl <= msd_segs;
    if (!fits) {   // an overrun (the caller regrows) or an unexpected shape
        HIP_TRY(launch_round_tail(r, 1, s, false, &E.prof));
        return HSS_OK;
    }
    const uint64_t need = 4 * m + nivl + 1;
    if (need > E.psort_cap) {
        if (E.psort_mem) dev_release(E.mem, E.psort_mem);
        E.psort_mem = nullptr;
        E.psort_cap = 0;
        const uint64_t want = need + need / 4;
        HIP_TRY(dev_alloc(E.mem, &E.psort_mem, want * sizeof(uint64_t)));
        E.psort_cap = want;
    }
    uint64_t* x0 = (uint64_t*)E.psort_mem;
    uint64_t* x1 = x0 + m;
    uint64_t* y0 = x1 + m;
    uint64_t* y1 = y0 + m;
    uint64_t* off = y1 + m;
    HIP_TRY(launch_probe_offsets(r, off, s));
    HybridSort hs;
    hs.key_bytes = 8;
    hs.seg_off = off;
    hs.num_segs = nivl;
    hs.max_seg_len = m;
    hs.total_len = m;
    hs.counts = E.counts;
    hs.sb_start = E.sb_start;
    hs.sb_len = E.sb_len;
    hs.ov = E.ov;
    hs.ov2 = E.ov2;
    hs.eq = E.eq;
    hs.lw = E.lw;
    hs.pj = E.pj;
    hs.sl = E.sl;
    hs.has_payload = true;
    hs.keys_tmp = y0;
    hs.vals_tmp = y1;
    // by tag (tags are distinct) ...
    hs.keys_in = r.g_tag;
    hs.vals_in = r.g_key;
    hs.keys_out = x0;
    hs.vals_out = x1;
    HIP_TRY(hybrid_sort(hs, s, E.hh));
    // ... then stably by key: (key, tag) order
    hs.keys_in = x1;
    hs.vals_in = x0;
    hs.keys_out = r.ps_key;
    hs.vals_out = r.ps_tag;
    HIP_TRY(hybrid_sort(hs, s, E.hh));
    HIP_TRY(launch_probe_finish(r, s));
    // more probes than fences in a segment: rank against the keys in LDS
    r.dense_rank = m * kFenceStride >= E.max_seg ? 1u : 0u;
    const hipError_t et = launch_round_tail(r, 1, s, true, &E.prof);
    r.dense_rank = 0;
    HIP_TRY(et);
    return HSS_OK;
}

// Rounds 1..n queued in one go: from a graph captured once for the engine's
// current probe and count-matrix buffers (on a stream of its own, so that
// the caller's stream may be any stream), replayed on the caller's stream.
hss_status launch_first_rounds(Engine& E, uint32_t n, hipStream_t s) {
    RoundArgs& r = E.ra;
    if (E.tune.plain_launches || E.own_stream) {
        for (uint32_t j = 1; j <= n; ++j) HIP_TRY(launch_round(r, j, s, &E.prof));
        return HSS_OK;
    }
    if (!E.rounds_exec || E.rounds_exec_n != n || E.rounds_exec_cap != E.cap || E.rounds_exec_cm != E.cm_cap ||
        E.rounds_exec_knobs != E.knob_gen) {
        if (E.rounds_exec) HIP_TRY(hipGraphExecDestroy(E.rounds_exec));
        E.rounds_exec = nullptr;
        if (!E.capture_stream) HIP_TRY(hipStreamCreateWithFlags(&E.capture_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(E.capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (uint32_t j = 1; j <= n && le == hipSuccess; ++j) le = launch_round(r, j, E.capture_stream, nullptr);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(E.capture_stream, &g);
        HIP_TRY(le);
        HIP_TRY(ce);
        const hipError_t ie = hipGraphInstantiate(&E.rounds_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_TRY(ie);
        E.rounds_exec_n = n;
        E.rounds_exec_cap = E.cap;
        E.rounds_exec_cm = E.cm_cap;
        E.rounds_exec_knobs = E.knob_gen;
    }
    HIP_TRY(hipGraphLaunch(E.rounds_exec, s));
    return HSS_OK;
}

// The count matrix of a one-instance round as the trace reports it: c_s(e)
// at [e p + s] (the device keeps it segment-major, c_s(e) at [s m + e]).
std::vector<uint32_t> counts_probe_major(const std::vector<uint32_t>& cm, uint64_t m, uint64_t p) {
    std::vector<uint32_t> out(m * p);
    for (uint64_t s = 0; s < p; ++s)
        for (uint64_t e = 0; e < m; ++e) out[e * p + s] = cm[s * m + e];
    return out;
}

// The rounds after round j0 (0: from the start), until every splitter is
// settled.  With counters_ready the counters after round j0 were already
// read back (the rounds queued ahead of an exchange).
hss_status run_rounds(Engine& E, hipStream_t s, uint32_t j0, bool counters_ready) {
    RoundArgs& r = E.ra;
    const bool tracing = E.tune.trace_level >= 1;
    uint32_t restarts = 0;
    uint32_t j = j0;
    // the rounds that usually settle every splitter (k - 1 of them at the
    // configurations measured), queued in one go; each further round is
    // queued and read back on its own
    const uint32_t first_chunk = std::min(std::max(E.k_max, 2u) - 1, E.J);
    uint32_t chunk = tracing ? 1u : (j == 0 ? first_chunk : 1u);
    bool queue = !counters_ready;
    for (;;) {
        uint32_t stop = E.J;
        if (E.tune.max_rounds) stop = std::min(stop, E.tune.max_rounds);
        if (queue) {
            const uint32_t upto = std::min(j + chunk, stop);
            if (j == 0 && upto > 1 && !E.big_first) {
                const hss_status sg = launch_first_rounds(E, upto, s);
                if (sg != HSS_OK) return sg;
                j = upto;
            }
            while (j < upto) {
                ++j;
                if (j == 1 && E.big_first) {
                    const hss_status sb = big_first_round(E, s);
                    if (sb != HSS_OK) return sb;
                } else {
                    HIP_TRY(launch_round(r, j, s, &E.prof));
                }
            }
            hss_status st = read_counters(E, s, j);
            if (st != HSS_OK) return st;
        }
        queue = true;
        const RoundCounters c = *E.h_ctr;
        if (c.overflow) {
            if (++restarts > kMaxRestarts) return fail(HSS_ERR_DEVICE, "probe buffers keep overflowing");
            // the recorded needs, and at least twice what overflowed
            const bool probes_short = c.m_max > E.cap || c.cm_max <= E.cm_cap;
            const uint64_t need = probes_short ? std::max<uint64_t>(c.m_max + c.m_max / 4 + 1024, 2 * E.cap) : E.cap;
            const uint64_t cm_need = c.cm_max > E.cm_cap ? std::max<uint64_t>(c.cm_max + c.cm_max / 4, 2 * E.cm_cap) : E.cm_cap;
            hss_status st = grow(E, need, cm_need);
            if (st != HSS_OK) return st;
            E.trace.clear();
            HIP_TRY(launch_round_init(r, s));
            j = 0;
            chunk = tracing ? 1u : first_chunk;
            continue;
        }
        if (c.err) return fail(HSS_ERR_DEVICE, "device consistency check failed (code " + std::to_string(c.err) + ")");
        if (tracing && c.n_unsettled > 0) {
            RoundRecord rec;
            record_round(E, rec, j);
            const uint64_t m = c.m_stored;
            const uint32_t q = E.ih[0].q - 1;
            std::vector<uint32_t> settled;
            hss_status st;
            if ((st = d2h(rec.key, r.ps_key, m, s)) != HSS_OK) return st;
            if ((st = d2h(rec.tag, r.ps_tag, m, s)) != HSS_OK) return st;
            if ((st = d2h(rec.rank, r.pr_rank, m, s)) != HSS_OK) return st;
            if ((st = d2h(rec.lo, r.lrank + 1, q, s)) != HSS_OK) return st;
            if ((st = d2h(rec.hi, r.urank + 1, q, s)) != HSS_OK) return st;
            if ((st = d2h(rec.chi, r.chi + 1, q, s)) != HSS_OK) return st;
            if ((st = d2h(settled, r.settled + 1, q, s)) != HSS_OK) return st;
            std::vector<uint32_t> cm;
            const uint64_t p = E.ih[0].p;
            if (E.tune.trace_level >= 2 && (st = d2h(cm, E.cmat, m * p, s)) != HSS_OK) return st;
            HIP_TRY(hipStreamSynchronize(s));
            if (E.tune.trace_level >= 2) rec.counts = counts_probe_major(cm, m, p);
            rec.settled.resize(q);
            for (uint32_t i = 0; i < q; ++i) {
                rec.settled[i] = settled[i] ? 1 : 0;
                if (settled[i]) { rec.lo[i] = kNone; rec.hi[i] = kNone; }
            }
            E.trace.push_back(std::move(rec));
        }
        if (c.n_after == 0) {
            if (!tracing) record_history(E, j);
            return HSS_OK;
        }
        if (j >= stop) {
            if (E.tune.max_rounds && j >= E.tune.max_rounds)
                return fail(HSS_ERR_NOT_CONVERGED, "round cap reached with " + std::to_string(c.n_after) + " splitters unsettled");
            return fail(HSS_ERR_DEVICE, "splitters unsettled after the rate reached 1");
        }
        chunk = 1;
    }
}

// Splitter rounds of every instance on the locally sorted buffer B; leaves
// chi in chi_all and in every instance's offsets.  With `ahead`, the rounds
// that usually settle every splitter are queued without reading anything
// back; the call's closing read-back checks them (finish()), and what follows
// on the stream must do nothing unless they did.
hss_status determine_splitters(Engine& E, hipStream_t s, bool ahead) {
    RoundArgs& r = E.ra;
    E.trace.clear();
    E.ahead_rounds = 0;
    if (E.Q > 2 * (uint32_t)E.ih.size()) {
        HIP_TRY(launch_round_init(r, s));
        const uint32_t first_chunk = std::min(std::max(E.k_max, 2u) - 1, E.J);
        const uint32_t upto = E.tune.max_rounds ? std::min(first_chunk, E.tune.max_rounds) : first_chunk;
        if (ahead && upto > 1 && !E.big_first && E.tune.trace_level == 0) {
            const hss_status sg = launch_first_rounds(E, upto, s);
            if (sg != HSS_OK) return sg;
            E.ahead_rounds = upto;
        } else {
            const hss_status st = run_rounds(E, s, 0, false);
            if (st != HSS_OK) return st;
        }
    }
    HIP_TRY(launch_finalize(r, E.chi_all, s));
    return HSS_OK;
}

// The exchange of the engine's call: into the callers' outputs, or into A
// before the bucket sort.  Behind rounds queued ahead of their read-back it
// waits for them (the gate).
ExchangeArgs exchange_args(Engine& E, bool sort_buckets) {
    ExchangeArgs ex;
    ex.key_bytes = E.key_bytes;
    ex.B = E.B;
    ex.Bv = E.payload ? E.Bv : nullptr;
    ex.n_inst = (uint32_t)E.ih.size();
    ex.n_rows = E.Q;
    ex.p_max = E.p_max;
    ex.inst = E.inst_d;
    ex.run = E.run_d;
    ex.seg_off = E.seg_off;
    ex.row_inst = E.row_inst;
    ex.prow = E.ra.prow;
    ex.chi_all = E.chi_all;
    ex.dst = E.dst;
    ex.chunk0 = E.chunk0;
    ex.max_chunks = exchange_chunk_bound(E.n_tot, E.Q);
    ex.total = E.n_tot;
    ex.out = sort_buckets ? E.A : nullptr;
    ex.vout = sort_buckets ? E.Av : nullptr;
    ex.err = &E.ra.ctr->err;
    ex.prof = &E.prof;
    ex.gate = E.ahead_rounds ? E.ra.ctr : nullptr;
    return ex;
}

// One call on an engine: local sort, rounds, exchange (and, for one
// instance, the bucket sort).  The per-call records are already queued.
hss_status engine_run(Engine& E, const void* kin, const uint64_t* vin, void* kout, uint64_t* vout,
                      hipStream_t s, bool sort_buckets) {
    if (E.listed) {
        HIP_TRY(launch_segment_sources(E.ra, E.msd_seg, E.n_msd, E.msd_src,
                                       E.payload ? E.msd_vsrc : nullptr, E.key_bytes, s));
        HIP_TRY(launch_segment_sources(E.ra, E.direct_seg, E.n_direct, E.direct_src,
                                       E.payload ? E.direct_vsrc : nullptr, E.key_bytes, s));
    }
    if (E.pre_rounds) {
        // after the work already on the caller's stream (the previous call's
        // rounds read the masks)
        HIP_TRY(hipEventRecord(E.ev_start, s));
        HIP_TRY(hipStreamWaitEvent(E.aux, E.ev_start, 0));
        HIP_TRY(launch_presample_reset(E.pre_mem, kPreRounds, E.aux));
        for (uint32_t j = 1; j <= E.pre_rounds; ++j)
            HIP_TRY(launch_presample(E.cur_seed, E.n_tot, j, E.pre_thresh[j - 1],
                                     E.pre_mem + kPreRounds + (uint64_t)(j - 1) * E.pre_cap, E.pre_cap,
                                     E.pre_mem + (j - 1), E.aux));
        HIP_TRY(hipEventRecord(E.ev_pre, E.aux));
    }
    // phase 1: local sort of every segment into B, with its fences
    hss_status st = segment_sort(E, true, kin, vin, E.B, E.Bv, E.A, E.Av, E.seg_off, E.S, E.max_seg,
                                 E.first_shift, E.first_base, true, s);
    if (st != HSS_OK) return st;
    if (E.pre_rounds) HIP_TRY(hipStreamWaitEvent(s, E.ev_pre, 0));
    // phase 2: splitter rounds; a plain partition of one instance queues its
    // exchange right behind the rounds that usually settle every splitter,
    // and the call's closing read-back checks that they did
    E.prof.begin(s);
    const bool ahead = !sort_buckets && !E.chi_out_host && E.ih.size() == 1 && E.tune.trace_level == 0;
    st = determine_splitters(E, s, ahead);
    if (st != HSS_OK) return st;
    E.prof.end(kProfRounds, s, 0);
    if (E.chi_out_host) {
        HIP_TRY(hipMemcpyAsync(E.chi_out_host, E.chi_all, (size_t)E.Q * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(E.chi_ready, s));
    }
    // phase 3: exchange into the outputs (or into A before the bucket sort)
    ExchangeArgs ex = exchange_args(E, sort_buckets);
    // sort (one instance): the bucket sort takes its first MSD digit over each
    // bucket's key range, and the exchange counts those digits as it writes
    // the buckets (the count pass of the bucket sort's first level)
    const uint32_t q = E.ih[0].q;
    const bool counted = sort_buckets && q > 1 && !E.tune.lsd_only;
    if (sort_buckets && q > 1)
        HIP_TRY(launch_bucket_shift(q, E.key_bytes * 8, E.ra.s_key, E.bucket_shift, E.bucket_base, s));
    if (counted) {
        const uint64_t tps = tiles_of(E.max_bucket);
        HIP_TRY(launch_sort_count_reset(E.counts, (uint64_t)q * tps * 256, E.lw, q, s));
        ex.sort_counts = E.counts;
        ex.sort_tps = (uint32_t)tps;
        ex.sort_shift = E.bucket_shift;
        ex.sort_base = E.bucket_base;
        ex.sort_and = E.lw.and_mask;
        ex.sort_or = E.lw.or_mask;
    }
    HIP_TRY(launch_exchange(ex, s));
    // phase 4 (sort, one instance): stable sort of every bucket
    if (sort_buckets) {
        const uint8_t* shifts = q > 1 ? E.bucket_shift : nullptr;
        const uint64_t* bases = q > 1 ? E.bucket_base : nullptr;
        E.sort_counted = counted;
        st = segment_sort(E, false, E.A, E.Av, kout, vout, E.B, E.Bv, E.chi_all, q, E.max_bucket,
                          shifts, bases, false, s);
        E.sort_counted = false;
        if (st != HSS_OK) return st;
    }
    return HSS_OK;
}

hss_status check_io_raw(bool payload, int key_bytes, uint64_t n, uint32_t p, const void* kin,
                        const uint64_t* vin, const void* kout, const uint64_t* vout,
                        const uint64_t* offsets) {
    if (!kin || !kout) return fail(HSS_ERR_INVALID_ARG, "null key pointer");
    if (payload != (vin != nullptr) || payload != (vout != nullptr))
        return fail(HSS_ERR_INVALID_ARG, "payload pointers must be given iff the plan has a payload");
    const void* ptrs[] = {kin, vin, kout, vout, offsets};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(HSS_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
    const size_t kb = n * key_bytes, vb = n * 8, ob = ((size_t)p + 1) * 8;
    if (overlap(kin, kb, kout, kb) || overlap(kin, kb, vout, vb) || overlap(vin, vb, kout, kb) ||
        overlap(vin, vb, vout, vb) || overlap(offsets, ob, kin, kb) || overlap(offsets, ob, kout, kb) ||
        overlap(offsets, ob, vin, vb) || overlap(offsets, ob, vout, vb) || overlap(kout, kb, vout, vb))
        return fail(HSS_ERR_INVALID_ARG, "outputs overlap inputs or each other");
    return HSS_OK;
}

hss_status check_io(const Engine& E, const InstHost& h, const void* kin, const uint64_t* vin,
                    const void* kout, const uint64_t* vout, const uint64_t* offsets) {
    return check_io_raw(E.payload, E.key_bytes, h.n, h.q, kin, vin, kout, vout, offsets);
}

hss_status finish(Engine& E, hipStream_t s) {
    if (E.ahead_rounds) {
        // rounds queued ahead of the exchange: one read-back for both
        const uint32_t j = E.ahead_rounds;
        hss_status st = read_counters(E, s, j);
        if (st != HSS_OK) return st;
        const RoundCounters c = *E.h_ctr;
        if (!c.overflow && c.n_after == 0) {
            E.ahead_rounds = 0;
            if (c.err)
                return fail(HSS_ERR_DEVICE, "device consistency check failed (code " + std::to_string(c.err) + ")");
            record_history(E, j);
            return HSS_OK;
        }
        // splitters left (or a buffer overran): the exchange did nothing; go
        // on with the rounds, then exchange
        st = run_rounds(E, s, j, true);
        if (st != HSS_OK) return st;
        HIP_TRY(launch_finalize(E.ra, E.chi_all, s));
        HIP_TRY(launch_exchange(exchange_args(E, false), s));
        E.ahead_rounds = 0;
    }
    // the exchange checks that every bucket's pieces add up to its size
    hss_status st = read_counters(E, s);
    if (st != HSS_OK) return st;
    if (E.h_ctr->err)
        return fail(HSS_ERR_DEVICE, "device consistency check failed (code " + std::to_string(E.h_ctr->err) + ")");
    return HSS_OK;
}

void set_knobs(Engine& E, const hss_knobs& k) {
    E.knobs = k;
    E.ra.pair_rank_from = k.pair_rank_from;
    E.ra.sample_grid = k.sample_workgroups;
    E.ra.pair_grid = k.pair_rank_workgroups;
    ++E.knob_gen;
}

// The autotuner: `call` runs one whole call of the engine on the caller's
// input and returns after its work has completed.  A setting's time is the
// fastest of three calls (the first call after a change of knobs also
// captures the round graph again).  Each knob in turn tries its other
// candidate values (the others at their best so far); the incumbent is timed
// again just before every candidate, so that a slow drift of the machine
// does not decide, and a candidate replaces it only when it is faster by more
// than kTuneMargin.  Every run writes the same outputs, so the call's result
// does not depend on the search.
constexpr double kTuneMargin = 0.02;

template <typename F>
hss_status autotune(Engine& E, hipStream_t s, F call) {
    using Clock = std::chrono::steady_clock;
    auto measure = [&](const hss_knobs& k, double* ms) -> hss_status {
        set_knobs(E, k);
        double m = 1e300;
        for (int r = 0; r < 3; ++r) {
            HIP_TRY(hipStreamSynchronize(s));
            const auto t0 = Clock::now();
            const hss_status st = call();
            if (st != HSS_OK) return st;
            m = std::min(m, std::chrono::duration<double, std::milli>(Clock::now() - t0).count());
        }
        *ms = m;
        return HSS_OK;
    };
    auto value = [](const hss_knobs& k, int knob) -> uint32_t {
        return knob == 0 ? k.small_sort_cap
                         : knob == 1 ? k.sample_workgroups : knob == 2 ? k.pair_rank_from : k.pair_rank_workgroups;
    };
    hss_knobs best = E.knobs;
    const uint32_t cands[4][3] = {{2048, 4096, 0}, {512, 1024, 2048}, {2, 3, 64}, {4096, 8192, 16384}};
    for (int knob = 0; knob < 4; ++knob) {
        for (int c = 0; c < 3; ++c) {
            const uint32_t v = cands[knob][c];
            if (v == 0 || v == value(best, knob)) continue;
            hss_knobs k = best;
            if (knob == 0) k.small_sort_cap = v;
            if (knob == 1) k.sample_workgroups = v;
            if (knob == 2) k.pair_rank_from = v;
            if (knob == 3) k.pair_rank_workgroups = v;
            double inc_ms = 0, ms = 0;
            hss_status st = measure(best, &inc_ms);
            if (st == HSS_OK) st = measure(k, &ms);
            if (st != HSS_OK) return st;
            if (ms < inc_ms * (1.0 - kTuneMargin)) best = k;
        }
    }
    best.tuned = 1;
    set_knobs(E, best);
    return call();   // the call's outputs, with the chosen knobs
}

hss_status run_plain(hss_plan_s* P, uint64_t seed, const void* kin, const uint64_t* vin, void* kout,
                     uint64_t* vout, uint64_t* d_offsets, void* stream, bool sort_buckets) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    Engine& E = P->e;
    hss_status st = check_io(E, E.ih[0], kin, vin, kout, vout, d_offsets);
    if (st != HSS_OK) return st;
    if (!d_offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets pointer");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(E.device));
    InstRun run{seed, kin, vin, kout, vout, d_offsets};
    E.cur_seed = seed;
    auto call = [&]() -> hss_status {
        HIP_TRY(launch_set_run(run, E.run_d, s));
        HIP_TRY(launch_counters_reset(E.ra.ctr, s));
        const hss_status r = engine_run(E, kin, vin, kout, vout, s, sort_buckets);
        if (r != HSS_OK) return r;
        return finish(E, s);
    };
    if (E.tune.autotune && !E.knobs.tuned) return autotune(E, s, call);
    return call();
}

hss_status new_engine_instance(Engine& E, uint64_t n, uint32_t p, double eps, uint32_t q = 0) {
    if (n == 0 || p == 0 || (uint64_t)p > n) return fail(HSS_ERR_INVALID_ARG, "need 1 <= p <= N");
    if (!(eps > 0.0 && eps < 1.0)) return fail(HSS_ERR_INVALID_ARG, "need 0 < eps < 1");
    if (q == 0) q = p;
    if (q > p) return fail(HSS_ERR_INVALID_ARG, "need 1 <= q <= p");
    InstHost h;
    h.n = n;
    h.p = p;
    h.q = q;
    h.eps = eps;
    instance_constants(h, E.tune);
    E.ih.push_back(h);
    return HSS_OK;
}

}  // namespace


// ------------------------------------------------------------- server ----

namespace {

double clock_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device and pinned blocks kept between batches: a released block is handed
// out again to the smallest request it covers without wasting more than
// half of it (plus 64 MiB); only a miss allocates.  The device bytes held
// (blocks in use plus idle ones) are kept within `limit`: idle blocks are
// freed, largest first, before an allocation would go over it and after a
// release leaves the total over it (blocks in use are never taken back, so
// the total exceeds the limit only while they alone do).
struct BlockCache : MemSource {
    std::mutex mu;
    std::multimap<size_t, void*> dev_free, host_free;
    std::unordered_map<void*, size_t> dev_size, host_size;
    size_t limit = ~size_t(0);
    size_t held = 0, max_held = 0;     // device bytes allocated by the cache

    static bool fits(size_t have, size_t want) { return have >= want && have <= 2 * want + (64u << 20); }

    // frees idle blocks, largest first, until `held + extra` is within the
    // limit or nothing idle is left (called with the lock held)
    void trim(size_t extra) {
        while (held + extra > limit && !dev_free.empty()) {
            auto it = std::prev(dev_free.end());
            (void)hipFree(it->second);
            dev_size.erase(it->second);
            held -= it->first;
            dev_free.erase(it);
        }
    }

    hipError_t dev_get(void** p, size_t bytes) override {
        std::lock_guard<std::mutex> g(mu);
        auto it = dev_free.lower_bound(bytes);
        if (it != dev_free.end() && fits(it->first, bytes)) {
            *p = it->second;
            dev_free.erase(it);
            return hipSuccess;
        }
        trim(bytes);
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipErrorOutOfMemory && !dev_free.empty()) {   // give back what is idle, then retry
            const size_t keep = limit;
            limit = 0;
            trim(0);
            limit = keep;
            (void)hipGetLastError();
            e = hipMalloc(p, bytes);
        }
        if (e == hipSuccess) {
            dev_size[*p] = bytes;
            held += bytes;
            max_held = std::max(max_held, held);
        }
        return e;
    }
    void dev_put(void* p) override {
        std::lock_guard<std::mutex> g(mu);
        dev_free.emplace(dev_size[p], p);
        trim(0);
    }
    hipError_t host_get(void** p, size_t bytes) override {
        std::lock_guard<std::mutex> g(mu);
        auto it = host_free.lower_bound(bytes);
        if (it != host_free.end() && fits(it->first, bytes)) {
            *p = it->second;
            host_free.erase(it);
            return hipSuccess;
        }
        hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
        if (e == hipSuccess) host_size[*p] = bytes;
        return e;
    }
    void host_put(void* p) override {
        std::lock_guard<std::mutex> g(mu);
        host_free.emplace(host_size[p], p);
    }
    ~BlockCache() override {
        for (auto& kv : dev_free) (void)hipFree(kv.second);
        for (auto& kv : host_free) (void)hipHostFree(kv.second);
    }
};

struct ServerReq {
    hss_request r{};
    double t_submit = 0, t_done = 0;
    hss_status st = HSS_OK;
    std::string msg;            // the worker's error message, for the caller's thread
    bool done = false;
};

}  // namespace

struct hss_server_s {
    int device = 0;
    uint64_t max_keys = 0;
    uint32_t max_reqs = 0;
    uint64_t budget = 0;
    double wait_s = 0;                  // a lone partition request's wait for company
    BlockCache cache;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, ServerReq> reqs;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;   // one per worker
    uint64_t admitted = 0;              // footprint bytes of the batches running
    uint32_t running = 0;
    uint64_t batches = 0, served = 0, keys = 0, max_admitted = 0;
    uint32_t max_running = 0;
};

namespace {

// Budget bytes of a request: inputs and outputs, and the engine's share of its
// keys (two key and payload buffers, fences, per-segment tables).
uint64_t footprint(const hss_request& r) {
    const uint64_t w = (r.key_type == HSS_U32 ? 4u : 8u) + (r.vals_in ? 8u : 0u);
    return 4 * r.n * w + r.n / 2 + 12ull * ((uint64_t)r.p + 1) * r.p + (1ull << 20);
}

// One sort request, run like hss_sort of a plan of its shape on a worker's
// stream with memory from the cache.
hss_status run_server_sort(hss_server_s* S, hipStream_t stream, const hss_request& r) {
    std::unique_ptr<Engine> E(new (std::nothrow) Engine());
    if (!E) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
    E->key_bytes = r.key_type == HSS_U32 ? 4 : 8;
    E->payload = r.vals_in != nullptr;
    E->mem = &S->cache;
    E->own_stream = stream;
    hss_status st = new_engine_instance(*E, r.n, r.p, r.eps);
    if (st == HSS_OK) st = engine_init(*E);
    if (st != HSS_OK) return st;
    E->cur_seed = r.seed;
    HIP_TRY(launch_set_run(InstRun{r.seed, r.keys_in, r.vals_in, r.keys_out, r.vals_out, r.offsets}, E->run_d,
                           stream));
    HIP_TRY(launch_counters_reset(E->ra.ctr, stream));
    st = engine_run(*E, r.keys_in, r.vals_in, r.keys_out, r.vals_out, stream, true);
    if (st != HSS_OK) return st;
    return finish(*E, stream);   // synchronises the stream
}

// One batch of queued requests (same operation, key type and payload
// choice), run like hss_batch_partition on a worker's stream with memory from
// the cache; a sort request is a batch of its own.
hss_status run_server_batch(hss_server_s* S, hipStream_t stream, const std::vector<hss_request>& rq) {
    if (rq[0].op == HSS_OP_SORT) return run_server_sort(S, stream, rq[0]);
    std::unique_ptr<Engine> E(new (std::nothrow) Engine());
    if (!E) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
    E->batch = true;
    E->key_bytes = rq[0].key_type == HSS_U32 ? 4 : 8;
    E->payload = rq[0].vals_in != nullptr;
    E->mem = &S->cache;
    E->own_stream = stream;
    for (const hss_request& r : rq) {
        hss_status st = new_engine_instance(*E, r.n, r.p, r.eps);
        if (st != HSS_OK) return st;
    }
    hss_status st = engine_init(*E);
    if (st != HSS_OK) return st;
    for (size_t i = 0; i < rq.size(); ++i)
        E->h_run[i] = InstRun{rq[i].seed, rq[i].keys_in, rq[i].vals_in, rq[i].keys_out, rq[i].vals_out,
                              rq[i].offsets};
    HIP_TRY(hipMemcpyAsync(E->run_d, E->h_run, rq.size() * sizeof(InstRun), hipMemcpyHostToDevice, stream));
    HIP_TRY(launch_counters_reset(E->ra.ctr, stream));
    st = engine_run(*E, nullptr, nullptr, nullptr, nullptr, stream, false);
    if (st != HSS_OK) return st;
    return finish(*E, stream);   // synchronises the stream
}

// A worker: takes the head of the queue and the later queued requests of its
// class (operation, key type, payload choice) that the budget admits, in
// submission order and within the batch limits -- requests of other classes
// keep their places -- and runs them as one batch on its stream; the head
// waits while the batches already running leave it no room, unless none is
// running.
// Queued requests of the head's class (operation, key width, payload), at
// most 2 counted; called with the lock held.
uint32_t same_class_queued(const hss_server_s* S) {
    if (S->queue.empty()) return 0;
    const hss_request& f = S->reqs.at(S->queue.front()).r;
    uint32_t c = 0;
    for (uint64_t t : S->queue) {
        const hss_request& r = S->reqs.at(t).r;
        if (r.op == f.op && r.key_type == f.key_type && (r.vals_in != nullptr) == (f.vals_in != nullptr) && ++c >= 2)
            break;
    }
    return c;
}

void server_loop(hss_server_s* S, uint32_t wid) {
    (void)hipSetDevice(S->device);
    const hipStream_t stream = S->streams[wid];
    for (;;) {
        std::vector<uint64_t> tickets;
        std::vector<hss_request> rq;
        uint64_t fp_total = 0;
        bool more = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [S] {
                if (S->queue.empty()) return S->stop;
                const uint64_t fp = footprint(S->reqs[S->queue.front()].r);
                return S->running == 0 || S->admitted + fp <= S->budget;
            });
            if (S->queue.empty()) return;   // stopping, nothing left
            if (S->wait_s > 0 && !S->stop && S->reqs[S->queue.front()].r.op == HSS_OP_PARTITION &&
                same_class_queued(S) < 2) {
                // a lone partition request waits, up to wait_s after its
                // submission, for another of its class to share its batch
                const double left = S->reqs[S->queue.front()].t_submit + S->wait_s - clock_s();
                if (left > 0)
                    S->cv_work.wait_for(lk, std::chrono::duration<double>(left),
                                        [S] { return S->stop || S->queue.empty() || same_class_queued(S) >= 2; });
                if (S->queue.empty()) continue;   // another worker took it
            }
            const hss_request& f = S->reqs[S->queue.front()].r;
            const bool pay = f.vals_in != nullptr;
            const hss_key_type kt = f.key_type;
            const hss_op op = f.op;
            const uint32_t max_reqs = op == HSS_OP_SORT ? 1u : S->max_reqs;
            uint64_t total = 0;
            for (auto it = S->queue.begin(); it != S->queue.end() && rq.size() < max_reqs;) {
                const hss_request& r = S->reqs[*it].r;
                if (r.op != op || r.key_type != kt || (r.vals_in != nullptr) != pay) {
                    ++it;   // another class: keeps its place for a later batch
                    continue;
                }
                const uint64_t fp = footprint(r);
                if (!rq.empty() && (total + r.n > S->max_keys || S->admitted + fp_total + fp > S->budget)) break;
                total += r.n;
                fp_total += fp;
                rq.push_back(r);
                tickets.push_back(*it);
                it = S->queue.erase(it);
            }
            S->admitted += fp_total;
            S->running += 1;
            S->max_running = std::max(S->max_running, S->running);
            S->max_admitted = std::max(S->max_admitted, S->admitted);
            more = !S->queue.empty();
        }
        if (more) S->cv_work.notify_one();   // another worker may take the rest
        hss_status st;
        try {
            st = run_server_batch(S, stream, rq);
        } catch (...) {
            st = fail(HSS_ERR_DEVICE, "unexpected exception");
        }
        const double t = clock_s();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (size_t i = 0; i < tickets.size(); ++i) {
                ServerReq& q = S->reqs[tickets[i]];
                q.st = st;
                if (st != HSS_OK) q.msg = g_last_error;
                q.t_done = t;
                q.done = true;
                S->keys += q.r.n;
            }
            S->batches += 1;
            S->served += tickets.size();
            S->admitted -= fp_total;
            S->running -= 1;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();   // budget freed
    }
}

hss_status retire(hss_server_s* S, std::unordered_map<uint64_t, ServerReq>::iterator it,
                  hss_status* result, double* t_submit, double* t_done) {
    if (result) *result = it->second.st;
    if (it->second.st != HSS_OK) g_last_error = it->second.msg;
    if (t_submit) *t_submit = it->second.t_submit;
    if (t_done) *t_done = it->second.t_done;
    S->reqs.erase(it);
    return HSS_OK;
}

}  // namespace

namespace {

hss_status plan_args(uint64_t n, uint32_t p, uint32_t q, double eps, hss_key_type kt,
                     const hss_tuning* tuning) {
    if (n == 0 || p == 0 || (uint64_t)p > n) return fail(HSS_ERR_INVALID_ARG, "need 1 <= p <= N");
    if (q == 0 || q > p) return fail(HSS_ERR_INVALID_ARG, "need 1 <= q <= p");
    if (!(eps > 0.0 && eps < 1.0)) return fail(HSS_ERR_INVALID_ARG, "need 0 < eps < 1");
    if (kt != HSS_U32 && kt != HSS_U64) return fail(HSS_ERR_INVALID_ARG, "bad key type");
    if (tuning) {
        for (uint32_t x : tuning->reserved)
            if (x) return fail(HSS_ERR_INVALID_ARG, "reserved tuning fields must be zero");
        if (tuning->pick_sampler && !tuning->probes_per_round)
            return fail(HSS_ERR_INVALID_ARG, "pick_sampler needs probes_per_round > 0");
    }
    if (n >= (1ull << 32)) return fail(HSS_ERR_UNSUPPORTED, "N >= 2^32 is not supported");
    return HSS_OK;
}

}  // namespace

extern "C" {

hss_status hss_plan_buckets(hss_plan_t* out, uint64_t n, uint32_t p, uint32_t q, double eps,
                            hss_key_type kt, int with_payload, const hss_tuning* tuning) {
    try {
        if (!out) return fail(HSS_ERR_INVALID_ARG, "null plan pointer");
        *out = nullptr;
        const hss_status va = plan_args(n, p, q, eps, kt, tuning);
        if (va != HSS_OK) return va;
        hss_plan_s* P = new (std::nothrow) hss_plan_s();
        if (!P) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
        Engine& E = P->e;
        E.key_bytes = kt == HSS_U32 ? 4 : 8;
        E.payload = with_payload != 0;
        if (tuning) E.tune = *tuning;
        hss_status st = new_engine_instance(E, n, p, eps, q);
        if (st == HSS_OK) st = engine_init(E);
        if (st != HSS_OK) {
            delete P;
            return st;
        }
        *out = P;
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_plan(hss_plan_t* out, uint64_t n, uint32_t p, double eps, hss_key_type kt,
                    int with_payload, const hss_tuning* tuning) {
    if (out) *out = nullptr;
    if (p == 0) return fail(HSS_ERR_INVALID_ARG, "need 1 <= p <= N");
    return hss_plan_buckets(out, n, p, p, eps, kt, with_payload, tuning);
}

void hss_plan_destroy(hss_plan_t P) {
    if (!P) return;
    try {
        delete P;
    } catch (...) {
    }
}

size_t hss_workspace_bytes(hss_plan_t P) {
    return P ? P->e.arena_bytes + P->e.probe_bytes + P->e.cm_cap * 4 : 0;
}

hss_status hss_partition(hss_plan_t P, uint64_t seed, const void* kin, const uint64_t* vin,
                         void* kout, uint64_t* vout, uint64_t* d_offsets, void* stream) {
    try {
        return run_plain(P, seed, kin, vin, kout, vout, d_offsets, stream, false);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_sort(hss_plan_t P, uint64_t seed, const void* kin, const uint64_t* vin,
                    void* kout, uint64_t* vout, uint64_t* d_offsets, void* stream) {
    try {
        return run_plain(P, seed, kin, vin, kout, vout, d_offsets, stream, true);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_local_sort(hss_plan_t P, const void* kin, const uint64_t* vin, void* kout,
                          uint64_t* vout, void* stream) {
    try {
        if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
        Engine& E = P->e;
        hss_status st = check_io(E, E.ih[0], kin, vin, kout, vout, nullptr);
        if (st != HSS_OK) return st;
        HIP_TRY(hipSetDevice(E.device));
        return segment_sort(E, true, kin, vin, kout, vout, E.A, E.Av, E.seg_off, E.S, E.max_seg, nullptr,
                            nullptr, false, (hipStream_t)stream);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

}  // extern "C"

// ------------------------------------------------- fixed workspace ----
// hss_partition_static: the whole workspace of a call is carved out of one
// file-scope device array, so a call allocates no device or pinned memory.
// In host code `scratch` names a host-side stand-in, not the array: its
// device address is looked up once per device with hipGetSymbolAddress, and
// only that address is handed to kernels.

namespace {

constexpr size_t kStaticScratchBytes = (size_t)HSS_STATIC_SCRATCH_MIB << 20;
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;                         // one call at a time (all devices)
void* g_static_ptr[kStaticMaxDevices] = {};     // device address of scratch, per device
alignas(256) unsigned char g_static_host[64 << 10];   // host words of the call in progress

// Bump allocation from a fixed device region and a fixed host buffer;
// releases return nothing (the region is reused by the next call).
struct FixedArena : MemSource {
    char* dev = nullptr;
    size_t dev_cap = 0, dev_used = 0;
    char* host = nullptr;
    size_t host_cap = 0, host_used = 0;
    static hipError_t take(char* base, size_t cap, size_t* used, void** p, size_t bytes) {
        const size_t at = (*used + 255) & ~size_t(255);
        if (at > cap || bytes > cap - at) return hipErrorOutOfMemory;
        *p = base + at;
        *used = at + bytes;
        return hipSuccess;
    }
    hipError_t dev_get(void** p, size_t bytes) override { return take(dev, dev_cap, &dev_used, p, bytes); }
    void dev_put(void*) override {}
    hipError_t host_get(void** p, size_t bytes) override { return take(host, host_cap, &host_used, p, bytes); }
    void host_put(void*) override {}
};

// Device bytes a fixed-region call of this engine takes (its layout, probe
// buffers, count matrix and the deeper levels' count tables), computed on
// the host alone.
size_t fixed_bytes(Engine& E) {
    Layout L;
    build_layout(E, L);
    return workspace_estimate(E);
}

// A one-instance engine laid out for a fixed region (no growth beyond it,
// plain launches, no second stream).
hss_status fixed_shape(Engine& E, uint64_t n, uint32_t p, double eps, hss_key_type kt, bool payload) {
    hss_status st = plan_args(n, p, p, eps, kt, nullptr);
    if (st != HSS_OK) return st;
    E.key_bytes = kt == HSS_U32 ? 4 : 8;
    E.payload = payload;
    E.tune.plain_launches = 1;
    E.fixed_mem = true;
    return new_engine_instance(E, n, p, eps);
}

hss_status static_shape(Engine& E, uint64_t n, uint32_t p, double eps, hss_key_type kt, bool payload) {
    if (n > HSS_STATIC_MAX_KEYS || p > HSS_STATIC_MAX_BUCKETS)
        return fail(HSS_ERR_UNSUPPORTED, "hss_partition_static takes at most " + std::to_string(HSS_STATIC_MAX_KEYS) +
                                             " keys and " + std::to_string(HSS_STATIC_MAX_BUCKETS) + " buckets");
    hss_status st = fixed_shape(E, n, p, eps, kt, payload);
    if (st != HSS_OK) return st;
    if (fixed_bytes(E) > kStaticScratchBytes)
        return fail(HSS_ERR_UNSUPPORTED, "the call needs more than the fixed workspace of " +
                                             std::to_string(kStaticScratchBytes) + " bytes");
    return HSS_OK;
}

// One partition in a fixed device region (mem.dev set) and its host words.
hss_status fixed_call(FixedArena& mem, Engine& E, uint64_t seed, const void* kin, const uint64_t* vin, void* kout,
                      uint64_t* vout, uint64_t* d_offsets, hipStream_t s) {
    E.mem = &mem;
    E.own_stream = s;
    hss_status st = engine_init(E);
    if (st != HSS_OK) return st;
    E.cur_seed = seed;
    const InstRun run{seed, kin, vin, kout, vout, d_offsets};
    HIP_TRY(launch_set_run(run, E.run_d, s));
    HIP_TRY(launch_counters_reset(E.ra.ctr, s));
    st = engine_run(E, kin, vin, kout, vout, s, false);
    if (st != HSS_OK) return st;
    return finish(E, s);
}

}  // namespace

extern "C" {

hss_status hss_partition_static_bytes(uint64_t n, uint32_t p, double eps, hss_key_type kt, int with_payload,
                                      size_t* bytes, size_t* capacity) {
    try {
        Engine E;
        const hss_status st = static_shape(E, n, p, eps, kt, with_payload != 0);
        if (capacity) *capacity = kStaticScratchBytes;
        // a shape refused before it was laid out has no size
        if (bytes) *bytes = E.ih.empty() ? 0 : fixed_bytes(E);
        return st;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_partition_static(uint64_t n, uint32_t p, double eps, hss_key_type kt, uint64_t seed,
                                const void* kin, const uint64_t* vin, void* kout, uint64_t* vout,
                                uint64_t* d_offsets, void* stream) {
    try {
        const bool payload = vin != nullptr;
        hss_status st = check_io_raw(payload, kt == HSS_U32 ? 4 : 8, n, p, kin, vin, kout, vout, d_offsets);
        if (st != HSS_OK) return st;
        if (!d_offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets pointer");
        // shape and size checks on the host, before any device call
        FixedArena mem;
        Engine E;   // destroyed before mem
        st = static_shape(E, n, p, eps, kt, payload);
        if (st != HSS_OK) return st;
        std::lock_guard<std::mutex> lk(g_static_mu);
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        if (dev < 0 || dev >= kStaticMaxDevices) return fail(HSS_ERR_UNSUPPORTED, "device ordinal too large");
        if (!g_static_ptr[dev]) {
            // once per device, with that device current: the array's address
            // on it (each device holds its own copy)
            void* ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return fail(HSS_ERR_DEVICE, "no device address for the fixed workspace");
            g_static_ptr[dev] = ptr;
        }
        mem.dev = (char*)g_static_ptr[dev];
        mem.dev_cap = kStaticScratchBytes;
        mem.host = (char*)g_static_host;
        mem.host_cap = sizeof(g_static_host);
        return fixed_call(mem, E, seed, kin, vin, kout, vout, d_offsets, (hipStream_t)stream);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_partition_workspace_bytes(uint64_t n, uint32_t p, double eps, hss_key_type kt, int with_payload,
                                         size_t* bytes) {
    try {
        if (!bytes) return fail(HSS_ERR_INVALID_ARG, "null bytes pointer");
        *bytes = 0;
        Engine E;
        const hss_status st = fixed_shape(E, n, p, eps, kt, with_payload != 0);
        if (st != HSS_OK) return st;
        *bytes = fixed_bytes(E);
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_partition_ws(uint64_t n, uint32_t p, double eps, hss_key_type kt, uint64_t seed, const void* kin,
                            const uint64_t* vin, void* kout, uint64_t* vout, uint64_t* d_offsets,
                            void* d_workspace, size_t workspace_bytes, void* stream) {
    try {
        const bool payload = vin != nullptr;
        const int kb = kt == HSS_U32 ? 4 : 8;
        hss_status st = check_io_raw(payload, kb, n, p, kin, vin, kout, vout, d_offsets);
        if (st != HSS_OK) return st;
        if (!d_offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets pointer");
        if (!d_workspace || ((uintptr_t)d_workspace & 255))
            return fail(HSS_ERR_INVALID_ARG, "the workspace must be a 256-byte aligned device pointer");
        const size_t kbytes = n * (size_t)kb, vb = n * 8, ob = ((size_t)p + 1) * 8;
        if (overlap(d_workspace, workspace_bytes, kin, kbytes) || overlap(d_workspace, workspace_bytes, kout, kbytes) ||
            overlap(d_workspace, workspace_bytes, vin, vb) || overlap(d_workspace, workspace_bytes, vout, vb) ||
            overlap(d_workspace, workspace_bytes, d_offsets, ob))
            return fail(HSS_ERR_INVALID_ARG, "the workspace overlaps an input or output");
        // shape and size on the host, before any device call
        std::unique_ptr<unsigned char[]> host(new (std::nothrow) unsigned char[(64 << 10) + 256]);
        if (!host) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
        FixedArena mem;
        Engine E;   // destroyed before mem
        st = fixed_shape(E, n, p, eps, kt, payload);
        if (st != HSS_OK) return st;
        const size_t need = fixed_bytes(E);
        if (need > workspace_bytes)
            return fail(HSS_ERR_INVALID_ARG, "the workspace holds " + std::to_string(workspace_bytes) +
                                                 " bytes; the call needs " + std::to_string(need));
        mem.dev = (char*)d_workspace;
        mem.dev_cap = workspace_bytes;
        mem.host = (char*)(((uintptr_t)host.get() + 255) & ~(uintptr_t)255);
        mem.host_cap = 64 << 10;
        return fixed_call(mem, E, seed, kin, vin, kout, vout, d_offsets, (hipStream_t)stream);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_get_constants(hss_plan_t P, uint64_t* tol, uint32_t* k, double* a, uint32_t max_j,
                             uint32_t* thresh, uint32_t* all) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    const InstHost& h = P->e.ih[0];
    if (tol) *tol = h.tol;
    if (k) *k = h.k;
    if (a) *a = h.a;
    for (uint32_t j = 1; j <= max_j; ++j) {
        uint32_t t;
        int al;
        round_rate(h, P->e.tune, j, false, &t, &al);   // the schedule itself, without forcing
        if (thresh) thresh[j - 1] = t;
        if (all) all[j - 1] = (uint32_t)al;
    }
    return HSS_OK;
}

uint32_t hss_trace_rounds(hss_plan_t P) { return P ? (uint32_t)P->e.trace.size() : 0; }

hss_status hss_trace_round_info(hss_plan_t P, uint32_t j, uint64_t* domain, uint64_t* m,
                                uint32_t* thresh, uint32_t* all) {
    if (!P || j >= P->e.trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->e.trace[j];
    if (domain) *domain = r.domain;
    if (m) *m = r.m;
    if (thresh) *thresh = r.thresh;
    if (all) *all = r.all;
    return HSS_OK;
}

hss_status hss_trace_round_probes(hss_plan_t P, uint32_t j, uint64_t* keys, uint64_t* tags,
                                  uint64_t* ranks) {
    if (!P || j >= P->e.trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->e.trace[j];
    if (r.key.size() != r.m) return fail(HSS_ERR_INVALID_ARG, "round probes need trace_level >= 1");
    if (keys) std::memcpy(keys, r.key.data(), r.m * 8);
    if (tags) std::memcpy(tags, r.tag.data(), r.m * 8);
    if (ranks) std::memcpy(ranks, r.rank.data(), r.m * 8);
    return HSS_OK;
}

hss_status hss_trace_round_counts(hss_plan_t P, uint32_t j, uint32_t* counts) {
    if (!P || j >= P->e.trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->e.trace[j];
    if (r.counts.size() != r.m * P->e.ih[0].p) return fail(HSS_ERR_INVALID_ARG, "round counts need trace_level >= 2");
    if (counts && !r.counts.empty()) std::memcpy(counts, r.counts.data(), r.counts.size() * 4);
    return HSS_OK;
}

hss_status hss_trace_round_state(hss_plan_t P, uint32_t j, uint64_t* lo_rank, uint64_t* hi_rank,
                                 uint8_t* settled, uint64_t* chi) {
    if (!P || j >= P->e.trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->e.trace[j];
    const size_t q = P->e.ih[0].q - 1;
    if (r.settled.size() != q) return fail(HSS_ERR_INVALID_ARG, "round state needs trace_level >= 1");
    if (lo_rank) std::memcpy(lo_rank, r.lo.data(), q * 8);
    if (hi_rank) std::memcpy(hi_rank, r.hi.data(), q * 8);
    if (settled) std::memcpy(settled, r.settled.data(), q);
    if (chi) std::memcpy(chi, r.chi.data(), q * 8);
    return HSS_OK;
}

hss_status hss_trace_splitters(hss_plan_t P, uint64_t* chi, uint64_t* s_key, uint64_t* s_tag,
                               uint64_t* pieces) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    try {
        Engine& E = P->e;
        HIP_TRY(hipSetDevice(E.device));
        HIP_TRY(hipDeviceSynchronize());
        const uint64_t p = E.ih[0].p, q = E.ih[0].q, n = E.ih[0].n;
        std::vector<uint64_t> c(q + 1, 0), sk(q + 1, 0), st(q + 1, kNone);
        std::vector<uint32_t> pr((q + 1) * p, 0);
        if (q > 1) {
            HIP_TRY(hipMemcpy(c.data(), E.ra.chi, (q + 1) * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(sk.data(), E.ra.s_key, (q + 1) * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(st.data(), E.ra.s_tag, (q + 1) * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(pr.data(), E.ra.prow, (q + 1) * p * 4, hipMemcpyDeviceToHost));
        }
        c[0] = 0;
        c[q] = n;
        sk[0] = sk[q] = 0;
        st[0] = st[q] = kNone;
        std::vector<uint64_t> sb(p + 1);
        for (uint64_t i = 0; i <= p; ++i) sb[i] = (uint64_t)(((u128)i * n) / p);
        if (chi) std::memcpy(chi, c.data(), (q + 1) * 8);
        if (s_key) std::memcpy(s_key, sk.data(), (q + 1) * 8);
        if (s_tag) std::memcpy(s_tag, st.data(), (q + 1) * 8);
        if (pieces) {
            for (uint64_t b = 0; b <= q; ++b)
                for (uint64_t s = 0; s < p; ++s)
                    pieces[b * p + s] = b == 0 ? 0 : (b == q ? sb[s + 1] - sb[s] : pr[b * p + s]);
        }
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_profile(hss_plan_t P, int enable) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    P->e.prof.collect();
    P->e.prof.on = enable != 0;
    return HSS_OK;
}

hss_status hss_profile_reset(hss_plan_t P) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    P->e.prof.reset();
    return HSS_OK;
}

hss_status hss_profile_read(hss_plan_t P, uint32_t family, double* ms, uint64_t* launches,
                            uint64_t* bytes) {
    if (!P || family >= (uint32_t)kProfSlots) return fail(HSS_ERR_INVALID_ARG, "bad plan or family");
    Profiler& pr = P->e.prof;
    pr.collect();
    if (ms) *ms = pr.ms[family];
    if (launches) *launches = pr.launches[family];
    if (bytes) *bytes = pr.bytes[family];
    return HSS_OK;
}

// ------------------------------------------------------------- batches ----

hss_status hss_batch_plan(hss_batch_t* out, const hss_instance_shape* shapes, uint32_t count,
                          int with_payload, const hss_tuning* tuning) {
    try {
        if (!out) return fail(HSS_ERR_INVALID_ARG, "null batch pointer");
        *out = nullptr;
        if (!shapes || count == 0) return fail(HSS_ERR_INVALID_ARG, "need at least one instance");
        if (tuning) {
            for (uint32_t x : tuning->reserved)
                if (x) return fail(HSS_ERR_INVALID_ARG, "reserved tuning fields must be zero");
            if (tuning->lsd_only) return fail(HSS_ERR_UNSUPPORTED, "lsd_only is for single plans");
            if (tuning->trace_level) return fail(HSS_ERR_UNSUPPORTED, "traces are for single plans");
            if (tuning->pick_sampler) return fail(HSS_ERR_UNSUPPORTED, "pick_sampler is for single plans");
        }
        hss_batch_s* Bt = new (std::nothrow) hss_batch_s();
        if (!Bt) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
        Bt->where.resize(count);
        for (uint32_t i = 0; i < count; ++i) {
            const hss_instance_shape& sh = shapes[i];
            if (sh.key_type != HSS_U32 && sh.key_type != HSS_U64) {
                delete Bt;
                return fail(HSS_ERR_INVALID_ARG, "bad key type of instance " + std::to_string(i));
            }
            const int g = sh.key_type == HSS_U32 ? 0 : 1;
            if (!Bt->eng[g]) {
                Bt->eng[g] = new (std::nothrow) Engine();
                if (!Bt->eng[g]) {
                    delete Bt;
                    return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
                }
                Bt->eng[g]->batch = true;
                Bt->eng[g]->key_bytes = g == 0 ? 4 : 8;
                Bt->eng[g]->payload = with_payload != 0;
                if (tuning) Bt->eng[g]->tune = *tuning;
            }
            Engine& E = *Bt->eng[g];
            Bt->where[i] = {g, (uint32_t)E.ih.size()};
            hss_status st = new_engine_instance(E, sh.n, sh.p, sh.eps);
            if (st != HSS_OK) {
                const std::string msg = "instance " + std::to_string(i) + ": " + g_last_error;
                delete Bt;
                return fail(st, msg);
            }
        }
        for (int g = 0; g < 2; ++g) {
            if (!Bt->eng[g]) continue;
            hss_status st = engine_init(*Bt->eng[g]);
            if (st != HSS_OK) {
                delete Bt;
                return st;
            }
        }
        *out = Bt;
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

void hss_batch_destroy(hss_batch_t Bt) {
    if (!Bt) return;
    try {
        delete Bt;
    } catch (...) {
    }
}

size_t hss_batch_workspace_bytes(hss_batch_t Bt) {
    if (!Bt) return 0;
    size_t b = 0;
    for (Engine* E : Bt->eng)
        if (E) b += E->arena_bytes + E->probe_bytes + E->cm_cap * 4;
    return b;
}

hss_status hss_batch_partition(hss_batch_t Bt, const hss_instance_io* io, void* stream) {
    try {
        if (!Bt || !io) return fail(HSS_ERR_INVALID_ARG, "null batch or io");
        for (uint32_t i = 0; i < Bt->where.size(); ++i) {
            const Engine& E = *Bt->eng[Bt->where[i].first];
            const InstHost& h = E.ih[Bt->where[i].second];
            const hss_instance_io& x = io[i];
            if (!x.offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets of instance " + std::to_string(i));
            hss_status st = check_io(E, h, x.keys_in, x.vals_in, x.keys_out, x.vals_out, x.offsets);
            if (st != HSS_OK) return fail(st, "instance " + std::to_string(i) + ": " + g_last_error);
        }
        hipStream_t s = (hipStream_t)stream;
        // one engine's whole call on stream `es`; returns after its work has completed
        auto run_engine = [&](int g, hipStream_t es) -> hss_status {
            Engine* E = Bt->eng[g];
            HIP_TRY(hipSetDevice(E->device));
            for (uint32_t i = 0; i < Bt->where.size(); ++i) {
                if (Bt->where[i].first != g) continue;
                const hss_instance_io& x = io[i];
                E->h_run[Bt->where[i].second] = InstRun{x.seed, x.keys_in, x.vals_in, x.keys_out,
                                                        x.vals_out, x.offsets};
            }
            auto call = [&]() -> hss_status {
                HIP_TRY(hipMemcpyAsync(E->run_d, E->h_run, E->ih.size() * sizeof(InstRun),
                                       hipMemcpyHostToDevice, es));
                HIP_TRY(launch_counters_reset(E->ra.ctr, es));
                const hss_status r = engine_run(*E, nullptr, nullptr, nullptr, nullptr, es, false);
                if (r != HSS_OK) return r;
                return finish(*E, es);
            };
            return (E->tune.autotune && !E->knobs.tuned) ? autotune(*E, es, call) : call();
        };
        if (!(Bt->eng[0] && Bt->eng[1])) {
            const int g = Bt->eng[0] ? 0 : 1;
            return run_engine(g, s);
        }
        // both widths: the u64 engine on the side stream, after the caller's
        // work already queued on its stream (the inputs)
        Engine* E1 = Bt->eng[1];
        HIP_TRY(hipSetDevice(E1->device));
        if (!Bt->side) {
            HIP_TRY(hipStreamCreateWithFlags(&Bt->side, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&Bt->ev_in, hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(Bt->ev_in, s));
        HIP_TRY(hipStreamWaitEvent(Bt->side, Bt->ev_in, 0));
        hss_status st1 = HSS_OK;
        std::string msg1;
        std::thread side([&]() {
            try {
                st1 = run_engine(1, Bt->side);
            } catch (...) {
                st1 = fail(HSS_ERR_DEVICE, "unexpected exception");
            }
            if (st1 != HSS_OK) msg1 = g_last_error;
        });
        hss_status st0;
        try {
            st0 = run_engine(0, s);
        } catch (...) {
            st0 = fail(HSS_ERR_DEVICE, "unexpected exception");
        }
        side.join();
        if (st0 != HSS_OK) return st0;
        if (st1 != HSS_OK) return fail(st1, msg1);
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_batch_profile(hss_batch_t Bt, int enable) {
    if (!Bt) return fail(HSS_ERR_INVALID_ARG, "null batch");
    for (Engine* E : Bt->eng)
        if (E) {
            E->prof.collect();
            E->prof.on = enable != 0;
        }
    return HSS_OK;
}

hss_status hss_batch_profile_reset(hss_batch_t Bt) {
    if (!Bt) return fail(HSS_ERR_INVALID_ARG, "null batch");
    for (Engine* E : Bt->eng)
        if (E) E->prof.reset();
    return HSS_OK;
}

hss_status hss_batch_profile_read(hss_batch_t Bt, uint32_t family, double* ms, uint64_t* launches,
                                  uint64_t* bytes) {
    if (!Bt || family >= (uint32_t)kProfSlots) return fail(HSS_ERR_INVALID_ARG, "bad batch or family");
    double t = 0;
    uint64_t l = 0, b = 0;
    for (Engine* E : Bt->eng)
        if (E) {
            E->prof.collect();
            t += E->prof.ms[family];
            l += E->prof.launches[family];
            b += E->prof.bytes[family];
        }
    if (ms) *ms = t;
    if (launches) *launches = l;
    if (bytes) *bytes = b;
    return HSS_OK;
}

// -------------------------------------------------------------- server ----

hss_status hss_server_create(hss_server_t* out, const hss_server_config* cfg) {
    try {
        if (!out) return fail(HSS_ERR_INVALID_ARG, "null server pointer");
        *out = nullptr;
        hss_server_config c{};
        if (cfg) c = *cfg;
        if (c.max_batch_keys >= (1ull << 32)) return fail(HSS_ERR_INVALID_ARG, "max_batch_keys must be below 2^32");
        if (c.workers > 16) return fail(HSS_ERR_INVALID_ARG, "at most 16 workers");
        std::unique_ptr<hss_server_s> S(new (std::nothrow) hss_server_s());
        if (!S) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
        S->max_keys = c.max_batch_keys ? c.max_batch_keys : (1ull << 30);
        S->max_reqs = c.max_batch_requests ? c.max_batch_requests : 1024u;
        S->wait_s = c.batch_wait_us * 1e-6;
        S->budget = c.hbm_budget ? c.hbm_budget : (64ull << 30);
        S->cache.limit = S->budget;
        const uint32_t nw = c.workers ? c.workers : 2u;
        HIP_TRY(hipGetDevice(&S->device));
        for (uint32_t w = 0; w < nw; ++w) {
            // default priority; no implicit ordering with other streams
            hipStream_t st = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            S->streams.push_back(st);
        }
        for (uint32_t w = 0; w < nw; ++w) S->workers.emplace_back(server_loop, S.get(), w);
        *out = S.release();
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

uint64_t hss_server_footprint(const hss_request* req) { return req ? footprint(*req) : 0; }

void hss_server_destroy(hss_server_t S) {
    if (!S) return;
    try {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        for (std::thread& w : S->workers)
            if (w.joinable()) w.join();
        (void)hipSetDevice(S->device);
        for (hipStream_t st : S->streams) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
        delete S;
    } catch (...) {
    }
}

hss_status hss_server_submit(hss_server_t S, const hss_request* req, uint64_t* ticket) {
    try {
        if (!S || !req || !ticket) return fail(HSS_ERR_INVALID_ARG, "null server, request or ticket");
        const hss_request& r = *req;
        if (r.key_type != HSS_U32 && r.key_type != HSS_U64) return fail(HSS_ERR_INVALID_ARG, "bad key type");
        if (r.op != HSS_OP_PARTITION && r.op != HSS_OP_SORT) return fail(HSS_ERR_INVALID_ARG, "bad operation");
        if (r.n == 0 || r.p == 0 || (uint64_t)r.p > r.n) return fail(HSS_ERR_INVALID_ARG, "need 1 <= p <= N");
        if (r.n >= (1ull << 32)) return fail(HSS_ERR_UNSUPPORTED, "N must be below 2^32");
        if (!(r.eps > 0.0 && r.eps < 1.0)) return fail(HSS_ERR_INVALID_ARG, "need 0 < eps < 1");
        if (!r.offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets pointer");
        hss_status st = check_io_raw(r.vals_in != nullptr, r.key_type == HSS_U32 ? 4 : 8, r.n, r.p,
                                     r.keys_in, r.vals_in, r.keys_out, r.vals_out, r.offsets);
        if (st != HSS_OK) return st;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->stop) return fail(HSS_ERR_INVALID_ARG, "server is stopping");
            const uint64_t t = S->next_ticket++;
            ServerReq q;
            q.r = r;
            q.t_submit = clock_s();
            S->reqs.emplace(t, q);
            S->queue.push_back(t);
            *ticket = t;
        }
        S->cv_work.notify_one();
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_server_poll(hss_server_t S, uint64_t ticket, int* done, hss_status* result,
                           double* t_submit, double* t_done) {
    if (!S) return fail(HSS_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(HSS_ERR_INVALID_ARG, "unknown ticket");
    if (done) *done = it->second.done ? 1 : 0;
    if (!it->second.done) return HSS_OK;
    return retire(S, it, result, t_submit, t_done);
}

hss_status hss_server_wait(hss_server_t S, uint64_t ticket, hss_status* result, double* t_submit,
                           double* t_done) {
    if (!S) return fail(HSS_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(HSS_ERR_INVALID_ARG, "unknown ticket");
    S->cv_done.wait(lk, [&] { return it->second.done; });
    return retire(S, it, result, t_submit, t_done);
}

hss_status hss_server_cancel(hss_server_t S, uint64_t ticket, int* cancelled) {
    if (!S) return fail(HSS_ERR_INVALID_ARG, "null server");
    if (cancelled) *cancelled = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(ticket);
        if (it == S->reqs.end()) return fail(HSS_ERR_INVALID_ARG, "unknown ticket");
        auto q = std::find(S->queue.begin(), S->queue.end(), ticket);
        if (q == S->queue.end()) return HSS_OK;   // taken by a worker: it finishes
        S->queue.erase(q);
        ServerReq& r = it->second;
        r.st = HSS_ERR_CANCELLED;
        r.msg = "request cancelled";
        r.t_done = clock_s();
        r.done = true;
        if (cancelled) *cancelled = 1;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();   // a worker waiting for this request's company
    return HSS_OK;
}

double hss_server_clock(void) { return clock_s(); }

hss_status hss_server_stats(hss_server_t S, uint64_t* batches, uint64_t* requests, uint64_t* keys,
                            uint32_t* max_concurrent, uint64_t* max_admitted) {
    if (!S) return fail(HSS_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    if (batches) *batches = S->batches;
    if (requests) *requests = S->served;
    if (keys) *keys = S->keys;
    if (max_concurrent) *max_concurrent = S->max_running;
    if (max_admitted) *max_admitted = S->max_admitted;
    return HSS_OK;
}

hss_status hss_server_memory(hss_server_t S, uint64_t* held, uint64_t* max_held) {
    if (!S) return fail(HSS_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> g(S->cache.mu);
    if (held) *held = S->cache.held;
    if (max_held) *max_held = S->cache.max_held;
    return HSS_OK;
}

hss_status hss_plan_knobs(hss_plan_t P, hss_knobs* out) {
    if (!P || !out) return fail(HSS_ERR_INVALID_ARG, "null plan or output");
    *out = P->e.knobs;
    return HSS_OK;
}

hss_status hss_plan_set_knobs(hss_plan_t P, const hss_knobs* k) {
    if (!P || !k) return fail(HSS_ERR_INVALID_ARG, "null plan or knobs");
    if ((k->small_sort_cap != 2048 && k->small_sort_cap != 4096) || k->sample_workgroups == 0 ||
        k->sample_workgroups > 65536 || k->pair_rank_workgroups == 0 || k->pair_rank_workgroups > 65536 ||
        k->pair_rank_from == 0)
        return fail(HSS_ERR_INVALID_ARG, "knob out of range");
    set_knobs(P->e, *k);
    return HSS_OK;
}

hss_status hss_batch_knobs(hss_batch_t Bt, hss_key_type kt, hss_knobs* out) {
    if (!Bt || !out) return fail(HSS_ERR_INVALID_ARG, "null batch or output");
    const Engine* E = Bt->eng[kt == HSS_U32 ? 0 : 1];
    if (!E) return fail(HSS_ERR_INVALID_ARG, "no instance of that key type");
    *out = E->knobs;
    return HSS_OK;
}

// ------------------------------------------------------ two stages ----
// Section 5.3 with two stages: the p segments are first split into r
// buckets, one per group of p/r processors; every group then runs HSS on its
// bucket alone.  Stage 1 is a plan with q = r buckets writing into a staging
// buffer; stage 2 is a batch of the r group instances built for the group
// sizes of the call (its device blocks come from a cache kept by the plan),
// reading each group where stage 1 wrote it and writing the caller's output.

}  // extern "C"

struct hss_staged_s {
    hss_plan_s st1;                 // stage 1: N keys, p segments, r buckets
    BlockCache cache;               // device and pinned blocks of stage 2
    uint32_t p = 0, r = 0, pg = 0;
    uint64_t n = 0;
    double eps2 = 0;
    hss_tuning tune2{};
    void* T = nullptr;              // stage-1 output: N keys
    uint64_t* Tv = nullptr;         // and payload
    void* T2 = nullptr;             // sort: stage-2 output (N keys, payload),
    uint64_t* T2v = nullptr;        // allocated by the first sort
    uint32_t* sort_counts = nullptr;   // sort: count table of the final buckets
    uint64_t sort_words = 0;
    uint64_t* h_off = nullptr;      // sort: pinned copy of the p+1 final offsets
    uint64_t* chi1 = nullptr;       // r+1 group boundaries (device)
    uint64_t* off2 = nullptr;       // r x (p/r + 1): offsets of every group
    uint64_t* h_chi1 = nullptr;     // pinned copy of chi1
    hipEvent_t chi_ready = nullptr; // h_chi1 holds stage 1's group boundaries
    hipStream_t setup = nullptr;    // stage 2's table uploads, beside stage 1's exchange
    size_t bytes = 0;
    double t_stage[3] = {0, 0, 0};  // host clock of the last call: stage 1, set-up, stage 2
    ~hss_staged_s() {
        (void)hipSetDevice(st1.e.device);
        (void)hipDeviceSynchronize();
        for (void* q : {T, (void*)Tv, T2, (void*)T2v, (void*)sort_counts, (void*)chi1, (void*)off2})
            if (q) (void)hipFree(q);
        if (h_chi1) (void)hipHostFree(h_chi1);
        if (h_off) (void)hipHostFree(h_off);
        if (chi_ready) (void)hipEventDestroy(chi_ready);
        if (setup) (void)hipStreamDestroy(setup);
    }
};

namespace {

hss_status staged_stage2(hss_staged_s* P, uint64_t seed, void* kout, uint64_t* vout, hipStream_t s) {
    Engine& E1 = P->st1.e;
    std::unique_ptr<Engine> E(new (std::nothrow) Engine());
    if (!E) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
    E->batch = true;
    E->key_bytes = E1.key_bytes;
    E->payload = E1.payload;
    E->tune = P->tune2;
    E->device = E1.device;
    E->mem = &P->cache;
    // the layout's uploads go through the plan's own stream (engine_init
    // waits for them), so that they need not wait for stage 1's exchange
    E->own_stream = P->setup;
    const uint64_t* c = P->h_chi1;
    if (c[0] != 0 || c[P->r] != P->n) return fail(HSS_ERR_DEVICE, "stage 1 returned bad group offsets");
    for (uint32_t g = 0; g < P->r; ++g) {
        const uint64_t ng = c[g + 1] - c[g];
        if (c[g + 1] < c[g] || c[g + 1] > P->n) return fail(HSS_ERR_DEVICE, "stage 1 returned bad group offsets");
        if (ng < P->pg)
            return fail(HSS_ERR_UNSUPPORTED, "group " + std::to_string(g) + " holds " + std::to_string(ng) +
                                                 " keys, fewer than its " + std::to_string(P->pg) + " processors");
        hss_status st = new_engine_instance(*E, ng, P->pg, P->eps2);
        if (st != HSS_OK) return st;
    }
    const double t0 = clock_s();
    hss_status st = engine_init(*E);
    E->own_stream = s;
    if (st != HSS_OK) return st;
    const size_t kb = (size_t)E1.key_bytes;
    for (uint32_t g = 0; g < P->r; ++g) {
        const uint64_t o = c[g];
        E->h_run[g] = InstRun{(seed + 1 + g), (const char*)P->T + o * kb, P->Tv ? P->Tv + o : nullptr,
                              (char*)kout + o * kb, vout ? vout + o : nullptr,
                              P->off2 + (uint64_t)g * (P->pg + 1)};
    }
    HIP_TRY(hipMemcpyAsync(E->run_d, E->h_run, (size_t)P->r * sizeof(InstRun), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_counters_reset(E->ra.ctr, s));
    // every key of group g lies between the stage-1 splitter keys g and g+1:
    // the first local sort takes its MSD digit over that range, as the
    // bucket sort of a plan does
    if (E->listed && E->n_msd > 0) {
        HIP_TRY(launch_bucket_shift(P->r, E1.key_bytes * 8, E1.ra.s_key, E1.bucket_shift, E1.bucket_base, s));
        HIP_TRY(launch_entry_ranges(E->n_msd, E->msd_seg, E->seg_inst, E1.bucket_shift, E1.bucket_base,
                                    E->msd_shift, E->msd_base, s));
        E->first_shift = E->msd_shift;
        E->first_base = E->msd_base;
    }
    const double t1 = clock_s();
    st = engine_run(*E, nullptr, nullptr, nullptr, nullptr, s, false);
    if (st != HSS_OK) return st;
    st = finish(*E, s);
    P->t_stage[1] = t1 - t0;
    P->t_stage[2] = clock_s() - t1;
    return st;
}

}  // namespace

extern "C" {

hss_status hss_staged_plan(hss_staged_t* out, uint64_t n, uint32_t p, uint32_t groups, double eps1,
                           double eps2, hss_key_type kt, int with_payload, const hss_tuning* tuning) {
    try {
        if (!out) return fail(HSS_ERR_INVALID_ARG, "null plan pointer");
        *out = nullptr;
        if (groups == 0 || p == 0 || p % groups != 0)
            return fail(HSS_ERR_INVALID_ARG, "need groups >= 1 dividing p");
        if (!(eps2 > 0.0 && eps2 < 1.0)) return fail(HSS_ERR_INVALID_ARG, "need 0 < eps2 < 1");
        if (tuning && (tuning->trace_level || tuning->lsd_only || tuning->pick_sampler))
            return fail(HSS_ERR_UNSUPPORTED, "traces, lsd_only and pick_sampler are for single plans");
        hss_status st = plan_args(n, p, groups, eps1, kt, tuning);
        if (st != HSS_OK) return st;
        std::unique_ptr<hss_staged_s> P(new (std::nothrow) hss_staged_s());
        if (!P) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
        Engine& E = P->st1.e;
        E.key_bytes = kt == HSS_U32 ? 4 : 8;
        E.payload = with_payload != 0;
        if (tuning) E.tune = *tuning;
        st = new_engine_instance(E, n, p, eps1, groups);
        if (st == HSS_OK) st = engine_init(E);
        if (st != HSS_OK) return st;
        P->p = p;
        P->r = groups;
        P->pg = p / groups;
        P->n = n;
        P->eps2 = eps2;
        if (tuning) P->tune2 = *tuning;
        P->tune2.autotune = 0;
        const size_t kb = n * (size_t)E.key_bytes;
        HIP_TRY(hipMalloc(&P->T, kb));
        if (E.payload) HIP_TRY(hipMalloc((void**)&P->Tv, n * 8));
        HIP_TRY(hipMalloc((void**)&P->chi1, ((size_t)groups + 1) * 8));
        HIP_TRY(hipMalloc((void**)&P->off2, (size_t)groups * (P->pg + 1) * 8));
        HIP_TRY(hipHostMalloc((void**)&P->h_chi1, ((size_t)groups + 1) * 8, hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&P->chi_ready, hipEventDisableTiming));
        HIP_TRY(hipStreamCreateWithFlags(&P->setup, hipStreamNonBlocking));
        P->bytes = kb + (E.payload ? n * 8 : 0) + ((size_t)groups + 1) * 8 + (size_t)groups * (P->pg + 1) * 8;
        *out = P.release();
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

void hss_staged_destroy(hss_staged_t P) {
    if (!P) return;
    try {
        delete P;
    } catch (...) {
    }
}

size_t hss_staged_workspace_bytes(hss_staged_t P) {
    if (!P) return 0;
    size_t b = P->st1.e.arena_bytes + P->bytes;
    std::lock_guard<std::mutex> g(P->cache.mu);
    for (auto& kv : P->cache.dev_size) b += kv.second;
    return b;
}

}  // extern "C"

namespace {

hss_status staged_check(hss_staged_s* P, const void* d_keys_in, const uint64_t* d_vals_in, void* d_keys_out,
                        uint64_t* d_vals_out, uint64_t* d_offsets, uint64_t* d_groups) {
    Engine& E = P->st1.e;
    hss_status st = check_io_raw(E.payload, E.key_bytes, P->n, P->p, d_keys_in, d_vals_in, d_keys_out,
                                 d_vals_out, d_offsets);
    if (st != HSS_OK) return st;
    if (!d_offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets pointer");
    if (d_groups && !aligned16(d_groups)) return fail(HSS_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
    const size_t kb = P->n * (size_t)E.key_bytes, vb = P->n * 8, gb = ((size_t)P->r + 1) * 8,
                 ob = ((size_t)P->p + 1) * 8;
    if (d_groups && (overlap(d_groups, gb, d_keys_in, kb) || overlap(d_groups, gb, d_keys_out, kb) ||
                     overlap(d_groups, gb, d_vals_in, vb) || overlap(d_groups, gb, d_vals_out, vb) ||
                     overlap(d_groups, gb, d_offsets, ob)))
        return fail(HSS_ERR_INVALID_ARG, "outputs overlap inputs or each other");
    return HSS_OK;
}

// The two stages into (kout, vout); returns after the stream has completed.
hss_status staged_run(hss_staged_s* P, uint64_t seed, const void* d_keys_in, const uint64_t* d_vals_in,
                      void* kout, uint64_t* vout, uint64_t* d_offsets, uint64_t* d_groups, hipStream_t s) {
    Engine& E = P->st1.e;
    hss_status st = HSS_OK;
    const size_t gb = ((size_t)P->r + 1) * 8;
    HIP_TRY(hipSetDevice(E.device));
    const double t0 = clock_s();
    bool stage1_done = false;
    if (E.tune.autotune && !E.knobs.tuned) {
        // the first call tunes stage 1 through whole plain calls
        st = run_plain(&P->st1, seed, d_keys_in, d_vals_in, P->T, P->Tv, P->chi1, s, false);
        if (st != HSS_OK) return st;
        HIP_TRY(hipMemcpyAsync(P->h_chi1, P->chi1, ((size_t)P->r + 1) * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        stage1_done = true;
    } else {
        // the group boundaries come back as soon as the rounds end: stage
        // 2 is laid out on the host while stage 1's exchange still runs
        HIP_TRY(launch_set_run(InstRun{seed, d_keys_in, d_vals_in, P->T, P->Tv, P->chi1}, E.run_d, s));
        HIP_TRY(launch_counters_reset(E.ra.ctr, s));
        E.chi_out_host = P->h_chi1;
        E.chi_ready = P->chi_ready;
        E.cur_seed = seed;
        st = engine_run(E, d_keys_in, d_vals_in, P->T, P->Tv, s, false);
        E.chi_out_host = nullptr;
        E.chi_ready = nullptr;
        if (st != HSS_OK) return st;
        HIP_TRY(hipEventSynchronize(P->chi_ready));
    }
    P->t_stage[0] = clock_s() - t0;
    st = staged_stage2(P, seed, kout, vout, s);
    // stage 1's own checks (its exchange ran before stage 2 on the stream)
    if (!stage1_done) {
        const hss_status s1 = finish(E, s);
        if (s1 != HSS_OK) return s1;
    }
    if (st != HSS_OK) return st;
    HIP_TRY(launch_stage_offsets(P->chi1, P->off2, P->r, P->pg, P->n, d_offsets, s));
    if (d_groups) HIP_TRY(hipMemcpyAsync(d_groups, P->chi1, gb, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HSS_OK;
}

}  // namespace

extern "C" {

hss_status hss_staged_partition(hss_staged_t P, uint64_t seed, const void* d_keys_in,
                                const uint64_t* d_vals_in, void* d_keys_out, uint64_t* d_vals_out,
                                uint64_t* d_offsets, uint64_t* d_groups, void* stream) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    try {
        hss_status st = staged_check(P, d_keys_in, d_vals_in, d_keys_out, d_vals_out, d_offsets, d_groups);
        if (st != HSS_OK) return st;
        return staged_run(P, seed, d_keys_in, d_vals_in, d_keys_out, d_vals_out, d_offsets, d_groups,
                          (hipStream_t)stream);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_staged_sort(hss_staged_t P, uint64_t seed, const void* d_keys_in, const uint64_t* d_vals_in,
                           void* d_keys_out, uint64_t* d_vals_out, uint64_t* d_offsets, uint64_t* d_groups,
                           void* stream) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    try {
        Engine& E = P->st1.e;
        hss_status st = staged_check(P, d_keys_in, d_vals_in, d_keys_out, d_vals_out, d_offsets, d_groups);
        if (st != HSS_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        HIP_TRY(hipSetDevice(E.device));
        const size_t kb = P->n * (size_t)E.key_bytes;
        if (!P->T2) {
            HIP_TRY(hipMalloc(&P->T2, kb));
            if (E.payload) HIP_TRY(hipMalloc((void**)&P->T2v, P->n * 8));
            HIP_TRY(hipHostMalloc((void**)&P->h_off, ((size_t)P->p + 1) * 8, hipHostMallocDefault));
            P->bytes += kb + (E.payload ? P->n * 8 : 0);
        }
        // the two-stage partition into the second buffer
        st = staged_run(P, seed, d_keys_in, d_vals_in, P->T2, P->T2v, d_offsets, d_groups, s);
        if (st != HSS_OK) return st;
        // the final buckets' sizes bound the sort's tiles
        HIP_TRY(hipMemcpyAsync(P->h_off, d_offsets, ((size_t)P->p + 1) * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        uint64_t maxb = 0;
        for (uint32_t b = 0; b < P->p; ++b) {
            if (P->h_off[b + 1] < P->h_off[b] || P->h_off[b + 1] > P->n)
                return fail(HSS_ERR_DEVICE, "the two stages returned bad offsets");
            maxb = std::max(maxb, P->h_off[b + 1] - P->h_off[b]);
        }
        if (P->h_off[0] != 0 || P->h_off[P->p] != P->n) return fail(HSS_ERR_DEVICE, "the two stages returned bad offsets");
        const uint64_t words = radix_count_words(P->p, maxb) + 256;
        if (words > P->sort_words) {
            if (P->sort_counts) HIP_TRY(hipFree(P->sort_counts));
            P->sort_counts = nullptr;
            P->sort_words = 0;
            HIP_TRY(hipMalloc((void**)&P->sort_counts, words * 4));
            P->sort_words = words;
        }
        // stable sort of every final bucket into the caller's output, through
        // stage 1's engine (its lists and tables serve p segments of N keys)
        // with the plan's count table and stage 1's output as the MSD buffer
        uint32_t* const keep = E.counts;
        const uint64_t keep_words = E.counts_words;
        E.counts = P->sort_counts;
        E.counts_words = P->sort_words;
        st = segment_sort(E, false, P->T2, P->T2v, d_keys_out, d_vals_out, P->T, P->Tv, d_offsets, P->p, maxb,
                          nullptr, nullptr, false, s);
        E.counts = keep;
        E.counts_words = keep_words;
        if (st != HSS_OK) return st;
        HIP_TRY(hipStreamSynchronize(s));
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_staged_times(hss_staged_t P, double* stage1_s, double* setup_s, double* stage2_s) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    if (stage1_s) *stage1_s = P->t_stage[0];
    if (setup_s) *setup_s = P->t_stage[1];
    if (stage2_s) *stage2_s = P->t_stage[2];
    return HSS_OK;
}

const char* hss_status_string(hss_status s) {
    switch (s) {
        case HSS_OK: return "ok";
        case HSS_ERR_INVALID_ARG: return "invalid argument";
        case HSS_ERR_UNSUPPORTED: return "unsupported";
        case HSS_ERR_OUT_OF_MEMORY: return "out of memory";
        case HSS_ERR_DEVICE: return "device error";
        case HSS_ERR_NOT_CONVERGED: return "not converged";
    }
    return "unknown status";
}

const char* hss_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
