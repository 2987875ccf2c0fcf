// libhss: plan, executor and C ABI of Histogram Sort with Sampling on one
// device.  The host drives the splitter rounds (one small read-back per
// round); every step on the data runs in the kernels of radix.hip,
// rounds.hip and exchange.hip.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "internal.hpp"

using namespace hss;

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

// largest per-round probe x segment count matrix kept on the device (words)
constexpr uint64_t kCountMatrixBudget = 1ull << 27;

struct RoundRecord {
    uint64_t domain = 0, m = 0;
    uint32_t thresh = 0, all = 0;
    std::vector<uint64_t> key, tag, rank;
    std::vector<uint64_t> lo, hi, chi;
    std::vector<uint8_t> settled;
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

}  // namespace

struct hss_plan_s {
    uint64_t n = 0;
    uint32_t p = 0;
    double eps = 0;
    int key_bytes = 8;
    bool payload = false;
    hss_tuning tune{};
    int device = 0;

    // constants (section 2 and section 4.2)
    uint64_t tol = 0;
    uint32_t k = 1;
    double a = 0;
    uint64_t max_seg = 0;      // ceil(N / p)
    uint64_t max_bucket = 0;   // ceil(N / p) + 2 tol

    // device memory
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void* B = nullptr;  uint64_t* Bv = nullptr;
    void* A = nullptr;  uint64_t* Av = nullptr;
    uint64_t* seg_off = nullptr;
    uint64_t* ideal = nullptr;
    uint32_t* counts = nullptr;
    RoundArgs ra{};
    uint32_t* dst = nullptr;
    RoundCounters* h_ctr = nullptr;   // pinned host copy

    // growable probe storage
    void* probe_mem = nullptr;
    size_t probe_bytes = 0;
    uint64_t cap = 0;
    void* sort_scratch = nullptr;
    size_t sort_scratch_bytes = 0;

    std::vector<RoundRecord> trace;
    Profiler prof;

    // per-probe segment counts of the current round (grown on demand)
    uint32_t* cmat = nullptr;
    uint64_t cmat_words = 0;
    uint8_t* bucket_shift = nullptr;
    uint64_t* bucket_base = nullptr;
    Fences fences;                    // of B, written by the local sort of hss_partition/hss_sort

    // hybrid sort state
    uint64_t* sb_start = nullptr;
    uint32_t* sb_len = nullptr;
    OversizeList ov;
    SlowList sl;
    HybridHost hh;
};

namespace {

void compute_constants(hss_plan_s& P) {
    const double nd = (double)P.n, pd = (double)P.p;
    P.tol = (uint64_t)std::floor((nd * P.eps) / (2.0 * pd));
    P.a = (2.0 * std::log(pd)) / P.eps;
    const double kk = std::ceil(std::log(P.a));
    P.k = (kk >= 1.0) ? (uint32_t)kk : 1u;
    if (P.tune.k_override) P.k = P.tune.k_override;
    P.max_seg = (P.n + P.p - 1) / P.p;
    P.max_bucket = P.max_seg + 2 * P.tol;
}

// Acceptance rule of round j: rate q_j = p s_j / N with s_j = a^(j/k),
// clamped at 1 ("take all").
void round_rate(const hss_plan_s& P, uint32_t j, bool forced, uint32_t* thresh, int* all) {
    const double s_j = std::pow(P.a, (double)j / (double)P.k);
    const double q = ((double)P.p * s_j) / (double)P.n;
    if (q >= 1.0 || (forced && j == 1 && P.tune.force_full_sample)) {
        *thresh = 0xFFFFFFFFu;
        *all = 1;
    } else {
        *thresh = (uint32_t)std::floor(q * 4294967296.0);
        *all = 0;
    }
}

size_t layout(hss_plan_s& P, char* base) {
    Arena ar;
    ar.base = base;
    const uint64_t n = P.n, p = P.p;
    P.B = ar.take<char>(n * P.key_bytes);
    P.A = ar.take<char>(n * P.key_bytes);
    P.Bv = P.payload ? ar.take<uint64_t>(n) : nullptr;
    P.Av = P.payload ? ar.take<uint64_t>(n) : nullptr;
    P.seg_off = ar.take<uint64_t>(p + 1);
    P.ideal = ar.take<uint64_t>(p + 1);
    P.counts = ar.take<uint32_t>(radix_count_words((uint32_t)p, P.max_bucket > P.max_seg ? P.max_bucket : P.max_seg));
    RoundArgs& r = P.ra;
    r.settled = ar.take<uint32_t>(p + 1);
    r.chi = ar.take<uint64_t>(p + 1);
    r.lrank = ar.take<uint64_t>(p + 1);
    r.urank = ar.take<uint64_t>(p + 1);
    r.s_key = ar.take<uint64_t>(p + 1);
    r.s_tag = ar.take<uint64_t>(p + 1);
    r.lpos = ar.take<uint32_t>((p + 1) * p);
    r.upos = ar.take<uint32_t>((p + 1) * p);
    r.prow = ar.take<uint32_t>((p + 1) * p);
    r.ivl_row = ar.take<uint32_t>(p);
    r.slices = ar.take<uint4>(p * p);
    r.ivl_nz = ar.take<uint32_t>(p + 1);
    r.ivl_tot = ar.take<uint64_t>(p + 1);
    r.ivl_dom = ar.take<uint64_t>(p);
    r.req_probe = ar.take<uint32_t>(2 * p);
    r.req_row = ar.take<uint32_t>(2 * p);
    r.req_kind = ar.take<uint32_t>(2 * p);
    r.ctr = ar.take<RoundCounters>(1);
    P.dst = (uint32_t*)r.slices;   // p x p words; the exchange runs after the last round
    P.fences.per_seg = (P.max_seg + kFenceStride - 1) / kFenceStride;
    P.fences.key = ar.take<uint64_t>(p * P.fences.per_seg);
    P.bucket_shift = ar.take<uint8_t>(p);
    P.bucket_base = ar.take<uint64_t>(p);
    P.sb_start = ar.take<uint64_t>(p * 256);
    P.sb_len = ar.take<uint32_t>(p * 256);
    const uint64_t ovc = oversize_capacity((uint32_t)p, n);
    P.ov.count = ar.take<uint32_t>(1);
    P.ov.tiles = ar.take<uint32_t>(1);
    P.ov.summary = ar.take<uint32_t>(4);
    P.ov.beg = ar.take<uint64_t>(ovc);
    P.ov.end = ar.take<uint64_t>(ovc);
    P.ov.base = ar.take<uint64_t>(ovc);
    P.ov.seg = ar.take<uint32_t>(ovc);
    P.ov.tile0 = ar.take<uint32_t>(ovc + 1);
    P.ov.tile_seg = ar.take<uint32_t>(oversize_tile_capacity((uint32_t)p, n));
    const uint64_t slc = slow_capacity((uint32_t)p, n);
    P.sl.count = ar.take<uint32_t>(1);
    P.sl.beg = ar.take<uint64_t>(slc);
    P.sl.len = ar.take<uint32_t>(slc);
    P.sl.bits = ar.take<uint8_t>(slc);
    P.sl.base = ar.take<uint64_t>(slc);
    P.sl.seg = ar.take<uint32_t>(slc);
    return ar.used;
}

hss_status grow_probes(hss_plan_s& P, uint64_t need) {
    if (need <= P.cap && P.probe_mem) return HSS_OK;
    uint64_t cap = P.cap ? P.cap : 4096;
    while (cap < need) cap *= 2;
    if (P.probe_mem) HIP_TRY(hipFree(P.probe_mem));
    P.probe_mem = nullptr;
    Arena ar;
    ar.base = nullptr;
    ar.take<uint64_t>(cap); ar.take<uint64_t>(cap); ar.take<uint32_t>(cap);
    ar.take<uint64_t>(cap); ar.take<uint64_t>(cap); ar.take<uint32_t>(cap);
    ar.take<uint64_t>(cap); ar.take<uint32_t>(cap); ar.take<uint32_t>(cap);
    P.probe_bytes = ar.used + 256;
    HIP_TRY(hipMalloc(&P.probe_mem, P.probe_bytes));
    ar.base = (char*)P.probe_mem;
    ar.used = 0;
    RoundArgs& r = P.ra;
    r.pr_key = ar.take<uint64_t>(cap);
    r.pr_tag = ar.take<uint64_t>(cap);
    r.pr_ivl = ar.take<uint32_t>(cap);
    r.ps_key = ar.take<uint64_t>(cap);
    r.ps_tag = ar.take<uint64_t>(cap);
    r.ps_ivl = ar.take<uint32_t>(cap);
    r.pr_rank = ar.take<uint64_t>(cap);
    r.pr_pos = ar.take<uint32_t>(cap);
    r.ps_seg = ar.take<uint32_t>(cap);
    r.cap = cap;
    P.cap = cap;
    return HSS_OK;
}

hss_status ensure_sort_scratch(hss_plan_s& P, uint64_t m) {
    const size_t need = probe_sort_scratch_bytes(m);
    if (need <= P.sort_scratch_bytes) return HSS_OK;
    if (P.sort_scratch) HIP_TRY(hipFree(P.sort_scratch));
    P.sort_scratch = nullptr;
    HIP_TRY(hipMalloc(&P.sort_scratch, need));
    P.sort_scratch_bytes = need;
    return HSS_OK;
}

bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

hss_status check_io(const hss_plan_s* P, const void* kin, const uint64_t* vin, const void* kout,
                    const uint64_t* vout, const uint64_t* offsets) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    if (!kin || !kout) return fail(HSS_ERR_INVALID_ARG, "null key pointer");
    if (P->payload != (vin != nullptr) || P->payload != (vout != nullptr))
        return fail(HSS_ERR_INVALID_ARG, "payload pointers must be given iff the plan has a payload");
    const void* ptrs[] = {kin, vin, kout, vout, offsets};
    for (const void* q : ptrs)
        if (q && !aligned16(q)) return fail(HSS_ERR_INVALID_ARG, "device pointers must be 16-byte aligned");
    const size_t kb = P->n * P->key_bytes, vb = P->n * 8, ob = (P->p + 1) * 8;
    if (overlap(kin, kb, kout, kb) || overlap(kin, kb, vout, vb) || overlap(vin, vb, kout, kb) ||
        overlap(vin, vb, vout, vb) || overlap(offsets, ob, kin, kb) || overlap(offsets, ob, kout, kb) ||
        overlap(offsets, ob, vin, vb) || overlap(offsets, ob, vout, vb) || overlap(kout, kb, vout, vb))
        return fail(HSS_ERR_INVALID_ARG, "outputs overlap inputs or each other");
    return HSS_OK;
}

hss_status read_counters(hss_plan_s& P, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(P.h_ctr, P.ra.ctr, sizeof(RoundCounters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HSS_OK;
}

template <typename T>
hss_status d2h(std::vector<T>& v, const T* d, size_t count, hipStream_t s) {
    v.resize(count);
    if (count) HIP_TRY(hipMemcpyAsync(v.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    return HSS_OK;
}

// Stable sort of the segments [seg_off[s], seg_off[s+1]) (the p input
// segments, or the p buckets after the exchange).
hss_status segment_sort(hss_plan_s& P, const void* kin, const uint64_t* vin, void* kout,
                        uint64_t* vout, void* ktmp, uint64_t* vtmp, const uint64_t* seg_off,
                        uint64_t max_len, const uint8_t* seg_shift, const uint64_t* seg_base,
                        const Fences* fences, hipStream_t s) {
    if (P.tune.lsd_only) {
        SegSort ss;
        ss.key_bytes = P.key_bytes;
        ss.keys_in = kin;
        ss.vals_in = vin;
        ss.keys_out = kout;
        ss.vals_out = vout;
        ss.keys_tmp = ktmp;
        ss.vals_tmp = vtmp;
        ss.seg_off = seg_off;
        ss.num_segs = P.p;
        ss.max_seg_len = max_len;
        ss.total_len = P.n;
        ss.counts = P.counts;
        ss.begin_bit = 0;
        ss.end_bit = P.key_bytes * 8;
        ss.prof = &P.prof;
        HIP_TRY(segmented_radix_sort(ss, s));
        return HSS_OK;
    }
    HybridSort hs;
    hs.key_bytes = P.key_bytes;
    hs.keys_in = kin;
    hs.vals_in = vin;
    hs.keys_out = kout;
    hs.vals_out = vout;
    hs.keys_tmp = ktmp;
    hs.vals_tmp = vtmp;
    hs.seg_off = seg_off;
    hs.num_segs = P.p;
    hs.max_seg_len = max_len;
    hs.total_len = P.n;
    hs.counts = P.counts;
    hs.sb_start = P.sb_start;
    hs.sb_len = P.sb_len;
    hs.seg_shift = seg_shift;
    hs.seg_base = seg_base;
    if (fences) hs.fences = *fences;
    hs.ov = P.ov;
    hs.sl = P.sl;
    hs.prof = &P.prof;
    HIP_TRY(hybrid_sort(hs, s, P.hh));
    return HSS_OK;
}

hss_status local_sort(hss_plan_s& P, const void* kin, const uint64_t* vin, void* kout,
                      uint64_t* vout, void* ktmp, uint64_t* vtmp, hipStream_t s) {
    return segment_sort(P, kin, vin, kout, vout, ktmp, vtmp, P.seg_off, P.max_seg, nullptr,
                        nullptr, nullptr, s);
}

// Splitter rounds on the locally sorted buffer P.B; leaves chi in d_offsets.
// Average keys per (interval, segment) slice below which the ranks are found
// by searching the slices instead of the fences.
constexpr uint64_t kNarrowSliceKeys = 8;

hss_status determine_splitters(hss_plan_s& P, uint64_t seed, uint64_t* d_offsets, hipStream_t s) {
    RoundArgs& r = P.ra;
    P.trace.clear();
    HIP_TRY(launch_round_init(r, s));
    for (uint32_t j = 1;; ++j) {
        uint32_t thresh;
        int all;
        round_rate(P, j, true, &thresh, &all);
        HIP_TRY(launch_intervals(r, s));
        HIP_TRY(launch_sample(r, seed, j, thresh, all, s));
        hss_status st = read_counters(P, s);
        if (st != HSS_OK) return st;
        const RoundCounters c = *P.h_ctr;
        if (c.err) return fail(HSS_ERR_DEVICE, "device consistency check failed (code " + std::to_string(c.err) + ")");
        if (c.n_unsettled == 0) break;
        if (P.tune.max_rounds && j > P.tune.max_rounds)
            return fail(HSS_ERR_NOT_CONVERGED, "round cap reached with " + std::to_string(c.n_unsettled) + " splitters unsettled");
        uint64_t m = c.m;
        if (m > P.cap) {   // resample into a larger buffer; the draw is a pure function of (seed, tag, round)
            st = grow_probes(P, m);
            if (st != HSS_OK) return st;
            HIP_TRY(launch_intervals(r, s));
            HIP_TRY(launch_sample(r, seed, j, thresh, all, s));
            st = read_counters(P, s);
            if (st != HSS_OK) return st;
            if (P.h_ctr->m != m) return fail(HSS_ERR_DEVICE, "probe count changed on resampling");
        }
        st = ensure_sort_scratch(P, m);
        if (st != HSS_OK) return st;
        HIP_TRY(launch_probe_sort(r, m, P.sort_scratch, P.sort_scratch_bytes, P.counts, s));
        // keep every probe's segment counts when they fit the budget, so the
        // locate step copies instead of searching again
        uint32_t* cmat = nullptr;
        const uint64_t words = m * (uint64_t)P.p;
        if (words <= kCountMatrixBudget) {
            if (words > P.cmat_words) {
                if (P.cmat) HIP_TRY(hipFree(P.cmat));
                P.cmat = nullptr;
                P.cmat_words = 0;
                uint64_t want = 1ull << 20;
                while (want < words) want *= 2;
                if (want > kCountMatrixBudget) want = kCountMatrixBudget;
                if (hipMalloc((void**)&P.cmat, want * 4) == hipSuccess) P.cmat_words = want;
                else P.cmat = nullptr;
            }
            if (P.cmat) cmat = P.cmat;
        }
        // Once the open intervals hold few keys per segment, a search inside
        // each probe's own interval slice reads fewer bytes than the fences
        // of every segment chunk.
        const Fences none;
        const bool narrow = j > 1 && c.n_ivl > 0 &&
                            c.domain <= kNarrowSliceKeys * (uint64_t)c.n_ivl * P.p;
        HIP_TRY(launch_rank(r, m, cmat, (P.tune.lsd_only || narrow) ? none : P.fences, P.max_seg, s));
        HIP_TRY(launch_settle(r, m, s));
        HIP_TRY(launch_locate(r, cmat, m, s));
        RoundRecord rec;
        rec.domain = c.domain;
        rec.m = m;
        rec.thresh = thresh;
        rec.all = (uint32_t)all;
        if (P.tune.trace_level >= 1) {
            const uint32_t q = P.p - 1;
            std::vector<uint32_t> settled;
            if ((st = d2h(rec.key, r.ps_key, m, s)) != HSS_OK) return st;
            if ((st = d2h(rec.tag, r.ps_tag, m, s)) != HSS_OK) return st;
            if ((st = d2h(rec.rank, r.pr_rank, m, s)) != HSS_OK) return st;
            if ((st = d2h(rec.lo, r.lrank + 1, q, s)) != HSS_OK) return st;
            if ((st = d2h(rec.hi, r.urank + 1, q, s)) != HSS_OK) return st;
            if ((st = d2h(rec.chi, r.chi + 1, q, s)) != HSS_OK) return st;
            if ((st = d2h(settled, r.settled + 1, q, s)) != HSS_OK) return st;
            HIP_TRY(hipStreamSynchronize(s));
            rec.settled.resize(q);
            for (uint32_t i = 0; i < q; ++i) {
                rec.settled[i] = settled[i] ? 1 : 0;
                if (settled[i]) { rec.lo[i] = kNone; rec.hi[i] = kNone; }
            }
        }
        P.trace.push_back(std::move(rec));
    }
    HIP_TRY(launch_finalize(r, d_offsets, s));
    return HSS_OK;
}

hss_status run(hss_plan_s* P, uint64_t seed, const void* kin, const uint64_t* vin, void* kout,
               uint64_t* vout, uint64_t* d_offsets, void* stream, bool sort_buckets) {
    hss_status st = check_io(P, kin, vin, kout, vout, d_offsets);
    if (st != HSS_OK) return st;
    if (!d_offsets) return fail(HSS_ERR_INVALID_ARG, "null offsets pointer");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(P->device));
    HIP_TRY(launch_counters_reset(P->ra.ctr, s));
    // phase 1: local sort of every segment into B, with its fences
    st = segment_sort(*P, kin, vin, P->B, P->Bv, P->A, P->Av, P->seg_off, P->max_seg, nullptr,
                      nullptr, P->tune.lsd_only ? nullptr : &P->fences, s);
    if (st != HSS_OK) return st;
    // phase 2: splitter rounds
    if (P->p == 1) {
        P->trace.clear();
        const uint64_t off[2] = {0, P->n};
        HIP_TRY(hipMemcpyAsync(d_offsets, off, sizeof(off), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        P->prof.begin(s);
        st = determine_splitters(*P, seed, d_offsets, s);
        if (st != HSS_OK) return st;
        P->prof.end(kProfRounds, s, 0);
    }
    // phase 3: exchange into the output (or into A before the bucket sort)
    ExchangeArgs ex;
    ex.key_bytes = P->key_bytes;
    ex.B = P->B;
    ex.Bv = P->Bv;
    ex.out = sort_buckets ? P->A : kout;
    ex.vout = sort_buckets ? P->Av : vout;
    ex.n = P->n;
    ex.p = P->p;
    ex.seg_off = P->seg_off;
    ex.prow = P->ra.prow;
    ex.chi = d_offsets;
    ex.dst = P->dst;
    ex.max_bucket = P->max_bucket;
    ex.err = &P->ra.ctr->err;
    ex.prof = &P->prof;
    HIP_TRY(launch_exchange(ex, s));
    // phase 4 (sort only): stable sort of every bucket
    if (sort_buckets) {
        const uint8_t* shifts = nullptr;
        const uint64_t* bases = nullptr;
        if (P->p > 1) {
            HIP_TRY(launch_bucket_shift(P->p, P->key_bytes * 8, P->ra.s_key, P->bucket_shift,
                                        P->bucket_base, s));
            shifts = P->bucket_shift;
            bases = P->bucket_base;
        }
        st = segment_sort(*P, P->A, P->Av, kout, vout, P->B, P->Bv, d_offsets, P->max_bucket,
                          shifts, bases, nullptr, s);
        if (st != HSS_OK) return st;
    }
    // the exchange checks that every bucket's pieces add up to its size
    st = read_counters(*P, s);
    if (st != HSS_OK) return st;
    if (P->h_ctr->err)
        return fail(HSS_ERR_DEVICE, "device consistency check failed (code " + std::to_string(P->h_ctr->err) + ")");
    return HSS_OK;
}

}  // namespace

extern "C" {

hss_status hss_plan(hss_plan_t* out, uint64_t n, uint32_t p, double eps, hss_key_type kt,
                    int with_payload, const hss_tuning* tuning) {
    try {
        if (!out) return fail(HSS_ERR_INVALID_ARG, "null plan pointer");
        *out = nullptr;
        if (n == 0 || p == 0 || (uint64_t)p > n)
            return fail(HSS_ERR_INVALID_ARG, "need 1 <= p <= N");
        if (!(eps > 0.0 && eps < 1.0)) return fail(HSS_ERR_INVALID_ARG, "need 0 < eps < 1");
        if (kt != HSS_U32 && kt != HSS_U64) return fail(HSS_ERR_INVALID_ARG, "bad key type");
        if (tuning) {
            for (uint32_t x : tuning->reserved)
                if (x) return fail(HSS_ERR_INVALID_ARG, "reserved tuning fields must be zero");
        }
        if (n >= (1ull << 32)) return fail(HSS_ERR_UNSUPPORTED, "N >= 2^32 is not supported");
        hss_plan_s* P = new (std::nothrow) hss_plan_s();
        if (!P) return fail(HSS_ERR_OUT_OF_MEMORY, "host allocation failed");
        P->n = n;
        P->p = p;
        P->eps = eps;
        P->key_bytes = kt == HSS_U32 ? 4 : 8;
        P->payload = with_payload != 0;
        if (tuning) P->tune = *tuning;
        compute_constants(*P);
        if (P->max_bucket >= (1ull << 32)) {
            delete P;
            return fail(HSS_ERR_UNSUPPORTED, "bucket bound >= 2^32");
        }
        hipError_t e = hipGetDevice(&P->device);
        if (e != hipSuccess) {
            delete P;
            return fail(HSS_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
        }
        P->arena_bytes = layout(*P, nullptr) + 256;
        e = hipMalloc(&P->arena, P->arena_bytes);
        if (e != hipSuccess) {
            delete P;
            return fail(HSS_ERR_OUT_OF_MEMORY, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
        }
        layout(*P, (char*)P->arena);
        e = hipHostMalloc((void**)&P->h_ctr, sizeof(RoundCounters) + 16, hipHostMallocDefault);
        if (e == hipSuccess) P->hh.pinned = (uint32_t*)((char*)P->h_ctr + sizeof(RoundCounters));
        if (e != hipSuccess) {
            (void)hipFree(P->arena);
            delete P;
            return fail(HSS_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
        }
        // segment boundaries floor(s N / p) and ideal ranks floor(i N / p): the
        // same integers (section 2)
        std::vector<uint64_t> sb(p + 1);
        for (uint64_t i = 0; i <= p; ++i) sb[i] = (uint64_t)(((u128)i * n) / p);
        RoundArgs& r = P->ra;
        r.key_bytes = P->key_bytes;
        r.B = P->B;
        r.n = n;
        r.p = p;
        r.seg_off = P->seg_off;
        r.ideal = P->ideal;
        r.tol = P->tol;
        e = hipMemcpy(P->seg_off, sb.data(), sb.size() * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(P->ideal, sb.data(), sb.size() * 8, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipHostFree(P->h_ctr);
            (void)hipFree(P->arena);
            delete P;
            return fail(HSS_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        // initial probe capacity: a generous multiple of the expected sample
        // p * s_j / s_{j-1} per round, grown on demand
        const double ratio = std::pow(P->a, 1.0 / P->k);
        uint64_t want = (uint64_t)(16.0 * p * (ratio > 1 ? ratio : 1)) + 65536;
        if (want > n) want = n;
        hss_status st = grow_probes(*P, want);
        if (st != HSS_OK) {
            (void)hipHostFree(P->h_ctr);
            (void)hipFree(P->arena);
            delete P;
            return st;
        }
        *out = P;
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

void hss_plan_destroy(hss_plan_t P) {
    if (!P) return;
    try {
        (void)hipSetDevice(P->device);
        (void)hipDeviceSynchronize();
        if (P->probe_mem) (void)hipFree(P->probe_mem);
        if (P->sort_scratch) (void)hipFree(P->sort_scratch);
        if (P->hh.fb_counts) (void)hipFree(P->hh.fb_counts);
        if (P->cmat) (void)hipFree(P->cmat);
        if (P->arena) (void)hipFree(P->arena);
        if (P->h_ctr) (void)hipHostFree(P->h_ctr);
        delete P;
    } catch (...) {
    }
}

size_t hss_workspace_bytes(hss_plan_t P) {
    return P ? P->arena_bytes + P->probe_bytes + P->sort_scratch_bytes : 0;
}

hss_status hss_partition(hss_plan_t P, uint64_t seed, const void* kin, const uint64_t* vin,
                         void* kout, uint64_t* vout, uint64_t* d_offsets, void* stream) {
    try {
        return run(P, seed, kin, vin, kout, vout, d_offsets, stream, false);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_sort(hss_plan_t P, uint64_t seed, const void* kin, const uint64_t* vin,
                    void* kout, uint64_t* vout, uint64_t* d_offsets, void* stream) {
    try {
        return run(P, seed, kin, vin, kout, vout, d_offsets, stream, true);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_local_sort(hss_plan_t P, const void* kin, const uint64_t* vin, void* kout,
                          uint64_t* vout, void* stream) {
    try {
        hss_status st = check_io(P, kin, vin, kout, vout, nullptr);
        if (st != HSS_OK) return st;
        HIP_TRY(hipSetDevice(P->device));
        return local_sort(*P, kin, vin, kout, vout, P->A, P->Av, (hipStream_t)stream);
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_get_constants(hss_plan_t P, uint64_t* tol, uint32_t* k, double* a, uint32_t max_j,
                             uint32_t* thresh, uint32_t* all) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    if (tol) *tol = P->tol;
    if (k) *k = P->k;
    if (a) *a = P->a;
    for (uint32_t j = 1; j <= max_j; ++j) {
        uint32_t t;
        int al;
        round_rate(*P, j, false, &t, &al);   // the schedule itself, without forcing
        if (thresh) thresh[j - 1] = t;
        if (all) all[j - 1] = (uint32_t)al;
    }
    return HSS_OK;
}

uint32_t hss_trace_rounds(hss_plan_t P) { return P ? (uint32_t)P->trace.size() : 0; }

hss_status hss_trace_round_info(hss_plan_t P, uint32_t j, uint64_t* domain, uint64_t* m,
                                uint32_t* thresh, uint32_t* all) {
    if (!P || j >= P->trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->trace[j];
    if (domain) *domain = r.domain;
    if (m) *m = r.m;
    if (thresh) *thresh = r.thresh;
    if (all) *all = r.all;
    return HSS_OK;
}

hss_status hss_trace_round_probes(hss_plan_t P, uint32_t j, uint64_t* keys, uint64_t* tags,
                                  uint64_t* ranks) {
    if (!P || j >= P->trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->trace[j];
    if (r.key.size() != r.m) return fail(HSS_ERR_INVALID_ARG, "round probes need trace_level >= 1");
    if (keys) std::memcpy(keys, r.key.data(), r.m * 8);
    if (tags) std::memcpy(tags, r.tag.data(), r.m * 8);
    if (ranks) std::memcpy(ranks, r.rank.data(), r.m * 8);
    return HSS_OK;
}

hss_status hss_trace_round_state(hss_plan_t P, uint32_t j, uint64_t* lo_rank, uint64_t* hi_rank,
                                 uint8_t* settled, uint64_t* chi) {
    if (!P || j >= P->trace.size()) return fail(HSS_ERR_INVALID_ARG, "no such round");
    const RoundRecord& r = P->trace[j];
    const size_t q = P->p - 1;
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
        HIP_TRY(hipSetDevice(P->device));
        HIP_TRY(hipDeviceSynchronize());
        const uint64_t p = P->p;
        std::vector<uint64_t> c(p + 1, 0), sk(p + 1, 0), st(p + 1, kNone);
        std::vector<uint32_t> pr((p + 1) * p, 0);
        if (p > 1) {
            HIP_TRY(hipMemcpy(c.data(), P->ra.chi, (p + 1) * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(sk.data(), P->ra.s_key, (p + 1) * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(st.data(), P->ra.s_tag, (p + 1) * 8, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(pr.data(), P->ra.prow, (p + 1) * p * 4, hipMemcpyDeviceToHost));
        }
        c[0] = 0;
        c[p] = P->n;
        sk[0] = sk[p] = 0;
        st[0] = st[p] = kNone;
        std::vector<uint64_t> sb(p + 1);
        for (uint64_t i = 0; i <= p; ++i) sb[i] = (uint64_t)(((u128)i * P->n) / p);
        if (chi) std::memcpy(chi, c.data(), (p + 1) * 8);
        if (s_key) std::memcpy(s_key, sk.data(), (p + 1) * 8);
        if (s_tag) std::memcpy(s_tag, st.data(), (p + 1) * 8);
        if (pieces) {
            for (uint64_t b = 0; b <= p; ++b)
                for (uint64_t s = 0; s < p; ++s)
                    pieces[b * p + s] = b == 0 ? 0 : (b == p ? sb[s + 1] - sb[s] : pr[b * p + s]);
        }
        return HSS_OK;
    } catch (...) {
        return fail(HSS_ERR_DEVICE, "unexpected exception");
    }
}

hss_status hss_profile(hss_plan_t P, int enable) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    P->prof.collect();
    P->prof.on = enable != 0;
    return HSS_OK;
}

hss_status hss_profile_reset(hss_plan_t P) {
    if (!P) return fail(HSS_ERR_INVALID_ARG, "null plan");
    P->prof.reset();
    return HSS_OK;
}

hss_status hss_profile_read(hss_plan_t P, uint32_t family, double* ms, uint64_t* launches,
                            uint64_t* bytes) {
    if (!P || family >= (uint32_t)kProfSlots) return fail(HSS_ERR_INVALID_ARG, "bad plan or family");
    P->prof.collect();
    if (ms) *ms = P->prof.ms[family];
    if (launches) *launches = P->prof.launches[family];
    if (bytes) *bytes = P->prof.bytes[family];
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
