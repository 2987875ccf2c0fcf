// Splitter rounds of HSS (section 4.2.2, steps 1-5) on the device, for any
// number of independent instances in the same launches.
//
// Round j, given the splitter state after round j-1, for every instance:
//   leaders  -- the distinct open intervals (L_i, U_i) of unsettled splitters
//               (identical intervals are taken once: they are either disjoint
//               or identical, section 4.2.2)
//   slices   -- per (interval, segment) the slice of the locally sorted
//               segment strictly inside the interval, as a run of 4-tag
//               Philox blocks of one flattened block space; the non-empty
//               slices are listed in (interval, segment) order
//   sample   -- every tag of the domain draws its Philox word and becomes a
//               probe when the word is below the instance's round threshold
//               (section 4.2.1: independent Bernoulli trials at rate p s_j/N)
//   group,   -- probes by interval; the intervals of an instance are disjoint
//   order       and in key order, so ranking (key, tag) inside each interval
//               sorts every instance's probes (the strict order of section 6.1)
//   rank     -- per probe and segment of its instance, the keys below it (the
//               local histograms), found from the segment's fences in LDS
//   reduce   -- R(e), the sum over the instance's segments (section 5.2)
//   settle   -- a probe in the target range settles splitter i (closest to
//               N i/p, lower rank on a tie); otherwise L and U move to the
//               closest probe ranks below and above N i/p
//               and the per-segment counts of every new bound or splitter
//               probe become the next round's slice ends and the piece
//               boundaries
// Every size (intervals, probes, work items) is read on the device, so a
// whole round is queued without waiting for the host, and a round with
// nothing left to do does nothing.  A capacity overrun sets a flag that turns
// the rest of the call into no-ops; the host then grows the buffers and runs
// the rounds again (the draws depend only on seed, tag and round).

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kT = 256;
// threads of the one-workgroup scans: kScanSmall up to kScanSmallRows rows
constexpr int kScanLarge = 1024;
constexpr int kScanSmall = 256;
constexpr uint32_t kScanSmallRows = 4096;
constexpr uint32_t kRankFences = kRankChunk / kFenceStride;
constexpr uint32_t kDenseTile = 4096;   // keys of a chunk staged at once by rank_dense_kernel
constexpr uint32_t kSampleStage = 256;  // probes a sampler wave stages in LDS (4 per lane)
constexpr uint32_t kReduceRows = 16;    // segments summed per reduction tile
constexpr uint32_t kReduceGrid = 2048;  // reduction workgroups (they stride over the tiles)
constexpr uint32_t kOrderLanes = 16;    // probes per ordering tile
constexpr uint32_t kOrderThreads = 512; // their comparisons split 32 ways (half a wave per probe)
constexpr uint32_t kOrderGrid = 1024;   // ordering workgroups (they stride over the tiles)

__device__ __forceinline__ bool halted(const RoundArgs& a) { return a.ctr->overflow != 0; }

// Exclusive scan of v[0, n) in place by one workgroup of kScanT threads
// (thread t scans a contiguous run serially); returns the total.
template <int kScanT, typename T>
__device__ uint64_t wg_scan_inplace(T* v, uint32_t n, uint64_t* scratch) {
    const uint32_t per = (n + kScanT - 1) / kScanT;
    const uint32_t r0 = min(threadIdx.x * per, n), r1 = min(r0 + per, n);
    uint64_t local = 0;
    for (uint32_t i = r0; i < r1; ++i) local += v[i];
    uint64_t tot;
    uint64_t run = block_exclusive_scan<uint64_t, kScanT>(local, scratch, &tot);
    for (uint32_t i = r0; i < r1; ++i) {
        const uint64_t x = v[i];
        v[i] = (T)run;
        run += x;
    }
    return tot;
}

// Last index i in [0, n) with v[i] <= x (v non-decreasing, v[0] <= x).
template <typename T>
__device__ __forceinline__ uint32_t last_le(const T* v, uint32_t n, uint64_t x) {
    uint32_t lo = 0, hi = n;   // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)v[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void counters_reset_kernel(RoundCounters* ctr) { *ctr = RoundCounters{}; }

__global__ void round_init_kernel(RoundArgs a) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < a.n_rows; r += gridDim.x * blockDim.x) {
        const InstDesc& D = a.inst[a.row_inst[r]];
        const uint32_t i = r - D.row0;
        a.settled[r] = (i == 0 || i == D.q) ? 1u : 0u;   // the ends are fixed
        a.chi[r] = 0;                                       // until the splitter settles
        a.lrank[r] = kNone;
        a.urank[r] = kNone;
        a.s_key[r] = 0;
        a.s_tag[r] = 0;
        a.l_tag[r] = 0;
        a.u_tag[r] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ctr = RoundCounters{};
}

// One workgroup: leaders of runs of identical unsettled intervals, in row
// order (instance by instance, splitter by splitter).
template <int kScanT>
__global__ __launch_bounds__(kScanT) void leaders_kernel(RoundArgs a, uint32_t round) {
    __shared__ uint32_t scratch[kScanT / kWave];
    if (halted(a)) {
        if (threadIdx.x == 0) { a.ctr->n_ivl = 0; a.ctr->n_unsettled = 0; }
        return;
    }
    const uint32_t Q = a.n_rows;
    const uint32_t per = (Q + kScanT - 1) / kScanT;
    const uint32_t r0 = min(threadIdx.x * per, Q), r1 = min(r0 + per, Q);
    // row 0 of every instance is a settled end, so an unsettled row r has r >= 1
    auto lead = [&](uint32_t r) {
        return a.settled[r] == 0 &&
               !(a.settled[r - 1] == 0 && a.lrank[r - 1] == a.lrank[r] && a.urank[r - 1] == a.urank[r]);
    };
    uint32_t nl = 0, nu = 0;
    for (uint32_t r = r0; r < r1; ++r) {
        nl += lead(r) ? 1u : 0u;
        nu += a.settled[r] == 0 ? 1u : 0u;
    }
    uint32_t tot;
    uint32_t o = block_exclusive_scan<uint32_t, kScanT>(nl, scratch, &tot);
    const uint32_t unsettled = block_sum<uint32_t, kScanT>(nu, scratch);
    for (uint32_t r = r0; r < r1; ++r) {
        if (lead(r)) {
            a.ivl_row[o] = r;
            a.ivl_inst[o] = a.row_inst[r];
            ++o;
        }
    }
    if (threadIdx.x == 0) {
        RoundCounters* c = a.ctr;
        a.hist[round - 1] = RoundHist{0, 0, unsettled, 0};
        c->n_ivl = tot;
        c->n_unsettled = unsettled;
        c->n_after = 0;
        c->m = 0;
        c->m_stored = 0;
        c->blocks = 0;
        c->domain = 0;
        c->n_slices = 0;
        c->tiles = 0;
        c->cm_need = 0;
    }
}

// Slice of segment s of instance D strictly inside the interval of its row i,
// as instance tags [ga, gb).
__device__ __forceinline__ void slice_bounds(const RoundArgs& a, const InstDesc& D, uint32_t i,
                                             uint32_t s, bool lnone, bool unone, uint64_t* ga,
                                             uint64_t* gb) {
    const uint32_t seg = D.seg0 + s;
    const uint64_t sb = a.seg_off[seg] - D.pos0;
    const uint64_t slen = a.seg_off[seg + 1] - a.seg_off[seg];
    const uint64_t lo = lnone ? 0 : a.lpos[D.tab0 + (uint64_t)i * D.p + s];
    const uint64_t hi = unone ? slen : a.upos[D.tab0 + (uint64_t)i * D.p + s];
    *ga = sb + lo;
    *gb = sb + (hi > lo ? hi : lo);
}

__device__ __forceinline__ uint64_t blocks_of(uint64_t ga, uint64_t gb) {
    return gb > ga ? ((gb - 1) >> 2) - (ga >> 2) + 1 : 0;
}

__device__ __forceinline__ uint64_t key_at(const RoundArgs& a, uint64_t i) {
    return a.key_bytes == 4 ? (uint64_t)((const uint32_t*)a.B)[i] : ((const uint64_t*)a.B)[i];
}

// Workgroup per interval k: Philox blocks, non-empty slices and tags of its
// slices, its bounds as (key, tag); clears its probe counters.
__global__ __launch_bounds__(kT) void slices_kernel(RoundArgs a) {
    __shared__ uint64_t scratch[kT / kWave];
    const uint32_t k = blockIdx.x;
    if (k >= a.ctr->n_ivl) return;
    const uint32_t row = a.ivl_row[k];
    const InstDesc D = a.inst[a.ivl_inst[k]];
    const uint32_t i = row - D.row0;
    const bool lnone = a.lrank[row] == kNone;
    const bool unone = a.urank[row] == kNone;
    uint64_t nb_sum = 0, nz_sum = 0, dom = 0;
    for (uint32_t s = threadIdx.x; s < D.p; s += kT) {
        uint64_t ga, gb;
        slice_bounds(a, D, i, s, lnone, unone, &ga, &gb);
        const uint64_t nb = blocks_of(ga, gb);
        nb_sum += nb;
        nz_sum += nb ? 1 : 0;
        dom += gb - ga;
    }
    nb_sum = block_sum<uint64_t, kT>(nb_sum, scratch);
    nz_sum = block_sum<uint64_t, kT>(nz_sum, scratch);
    dom = block_sum<uint64_t, kT>(dom, scratch);
    if (threadIdx.x == 0) {
        a.ivl_tot[k] = nb_sum;
        a.ivl_nz[k] = (uint32_t)nz_sum;
        a.ivl_dom[k] = dom;
        a.ivl_pcnt[k] = 0;
        a.ivl_cursor[k] = 0;
        a.ivl_lkey[k] = lnone ? 0ull : key_at(a, D.pos0 + a.l_tag[row]);
        a.ivl_ltag[k] = lnone ? -1ll : (int64_t)a.l_tag[row];
        a.ivl_ukey[k] = unone ? ~0ull : key_at(a, D.pos0 + a.u_tag[row]);
        a.ivl_utag[k] = unone ? INT64_MAX : (int64_t)a.u_tag[row];
    }
}

// One workgroup: exclusive scans of the interval block and slice totals.
template <int kScanT>
__global__ __launch_bounds__(kScanT) void ivl_scan_kernel(RoundArgs a) {
    __shared__ uint64_t scratch[kScanT / kWave];
    const uint32_t n = a.ctr->n_ivl;
    const uint64_t blocks = wg_scan_inplace<kScanT>(a.ivl_tot, n, scratch);
    const uint64_t slices = wg_scan_inplace<kScanT>(a.ivl_nz, n, scratch);
    // domain before every interval (an instance's domain is a difference)
    const uint64_t d = wg_scan_inplace<kScanT>(a.ivl_dom, n, scratch);
    if (threadIdx.x == 0) {
        a.ivl_tot[n] = blocks;
        a.ivl_nz[n] = (uint32_t)slices;
        a.ivl_dom[n] = d;
        a.ctr->blocks = blocks;
        a.ctr->n_slices = (uint32_t)slices;
        a.ctr->domain = d;
    }
}

// Workgroup per interval k: its non-empty slices, in segment order, into the
// slice list {first block in the flattened block space, first tag, end tag,
// interval}.  Blocks and slices of interval k start at the scanned offsets.
__global__ __launch_bounds__(kT) void compact_kernel(RoundArgs a) {
    __shared__ uint64_t scratch[kT / kWave];
    const uint32_t k = blockIdx.x;
    if (k >= a.ctr->n_ivl) return;
    const uint32_t row = a.ivl_row[k];
    const InstDesc D = a.inst[a.ivl_inst[k]];
    const uint32_t i = row - D.row0;
    const bool lnone = a.lrank[row] == kNone;
    const bool unone = a.urank[row] == kNone;
    uint64_t run = a.ivl_tot[k], run_nz = a.ivl_nz[k];
    for (uint32_t s0 = 0; s0 < D.p; s0 += kT) {
        const uint32_t s = s0 + threadIdx.x;
        uint64_t nb = 0, ga = 0, gb = 0;
        if (s < D.p) {
            slice_bounds(a, D, i, s, lnone, unone, &ga, &gb);
            nb = blocks_of(ga, gb);
        }
        uint64_t tot, tot_nz;
        const uint64_t pre = block_exclusive_scan<uint64_t, kT>(nb, scratch, &tot);
        const uint64_t pre_nz = block_exclusive_scan<uint64_t, kT>(nb ? 1 : 0, scratch, &tot_nz);
        if (nb) a.slices[run_nz + pre_nz] = make_uint4((uint32_t)(run + pre), (uint32_t)ga, (uint32_t)gb, k);
        run += tot;
        run_nz += tot_nz;
    }
}

// ivl_pcnt[k] += c for every lane of the wave (c = 0: nothing), with one
// atomic per distinct interval in the wave instead of one per probe (the
// probes of a round often share an interval, e.g. round 1's single one).
__device__ __forceinline__ void add_interval_counts(uint32_t* ivl_pcnt, uint32_t k, uint32_t c) {
    uint64_t rem = __ballot(c != 0);
    while (rem) {   // uniform
        const int leader = __ffsll((long long)rem) - 1;
        const uint32_t kk = (uint32_t)__shfl((int)k, leader);
        const uint64_t same = __ballot(c != 0 && k == kk);
        const uint32_t tot = wave_sum<uint32_t>((same & (1ull << lane_id())) ? c : 0u);
        if ((int)lane_id() == leader) atomicAdd(&ivl_pcnt[kk], tot);
        rem &= ~same;
    }
}

// Moves a wave's n staged probes to the probe arrays: one reservation, then
// the per-interval counts, one atomic per run of equal intervals in each
// 64-entry chunk (the wave's blocks walk the slices in interval order).
__device__ void flush_stage(const RoundArgs& a, const uint64_t* st_key, const uint32_t* st_tag,
                            const uint32_t* st_ivl, uint32_t n) {
    const uint32_t lane = lane_id();
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->m, (unsigned long long)n);
    base = shfl_u64(base, 0);
    if (base + n > a.cap && lane == 0) atomicOr(&a.ctr->overflow, 1u);
    for (uint32_t c0 = 0; c0 < n; c0 += kWave) {
        const uint32_t i = c0 + lane;
        const bool valid = i < n;
        uint32_t k = valid ? st_ivl[i] : 0u;
        if (valid && base + i < a.cap) {
            a.pr_key[base + i] = st_key[i];
            a.pr_tag[base + i] = st_tag[i];
            a.pr_ivl[base + i] = k;
        }
        // run starts: the chunk's first entry and every change of interval
        const bool start = valid && (lane == 0 || st_ivl[i - 1] != k);
        const uint64_t starts = __ballot(start);
        if (start) {
            const uint64_t later = lane + 1 < kWave ? starts >> (lane + 1) : 0ull;
            const uint32_t end = later ? lane + 1 + (uint32_t)(__ffsll((long long)later) - 1)
                                       : min((uint32_t)kWave, n - c0);
            // probes past the capacity count too: an overrun halts the rest
            // of the call, which the host repeats with larger buffers
            atomicAdd(&a.ivl_pcnt[k], end - lane);
        }
    }
}

// (key x, tag gx) before (key y, tag gy) in the order of section 6.1.
__device__ __forceinline__ bool key_tag_less(uint64_t x, int64_t gx, uint64_t y, int64_t gy) {
    return x < y || (x == y && gx < gy);
}

// Sampler of a round whose draws were taken ahead (one instance): thread per
// listed tag g.  g is a probe when (key, g) lies strictly inside an interval
// in the order (key, tag) -- the same as lying in the interval's slice of its
// segment, whose ends are the per-segment counts of the interval's bounds.
// The intervals are disjoint and in key order: the last one whose lower
// bound precedes (key, g) is the only one that may hold it.
template <typename K>
__device__ void sample_from_list(const RoundArgs& a, const uint32_t* list, uint32_t cnt) {
    const uint32_t n_ivl = a.ctr->n_ivl;
    if (n_ivl == 0) return;
    const InstDesc D = a.inst[0];
    const K* B = (const K*)a.B;
    const uint32_t lane = lane_id();
    const uint32_t stride = gridDim.x * blockDim.x;
    // whole waves step together (the probe slots are taken once per wave)
    for (uint32_t tb = blockIdx.x * blockDim.x + (threadIdx.x - lane); tb < cnt; tb += stride) {
        const uint32_t t = tb + lane;
        const uint64_t g = t < cnt ? list[t] : D.n;
        bool take = g < D.n;
        uint32_t kl = 0;
        uint64_t key = 0;
        if (take) {
            key = (uint64_t)B[D.pos0 + g];
            uint32_t lo = 0, hi = n_ivl;   // intervals whose lower bound precedes (key, g): [0, lo)
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (key_tag_less(a.ivl_lkey[mid], a.ivl_ltag[mid], key, (int64_t)g)) lo = mid + 1;
                else hi = mid;
            }
            take = lo > 0;
            if (take) {
                kl = lo - 1;
                take = key_tag_less(key, (int64_t)g, a.ivl_ukey[kl], a.ivl_utag[kl]);
            }
        }
        const uint64_t mask = __ballot(take);
        if (!mask) continue;   // uniform
        unsigned long long base = 0;
        const int leader = __ffsll((long long)mask) - 1;
        if ((int)lane == leader) base = atomicAdd(&a.ctr->m, (unsigned long long)__popcll(mask));
        base = shfl_u64(base, leader);
        bool stored = false;
        if (take) {
            const uint64_t o = base + __popcll(mask & lanes_below_mask());
            if (o < a.cap) {
                a.pr_key[o] = key;
                a.pr_tag[o] = g;
                a.pr_ivl[o] = kl;
                stored = true;
            } else {
                atomicOr(&a.ctr->overflow, 1u);
            }
        }
        add_interval_counts(a.ivl_pcnt, kl, stored ? 1u : 0u);
    }
}

// Wave-per-range sampler.  Wave w of W takes the blocks [w T / W, (w+1) T / W)
// of the flattened block space (T blocks), one block per lane per step.  The
// slice list is walked with a window of 64 consecutive entries, one per lane:
// slices are non-empty, so the 64 blocks of a step lie in the 64 slices that
// start with the slice of the step's first block, and the next step's first
// block lies at most one slice past the window.
template <typename K, bool kSingle>
__global__ __launch_bounds__(kT) void sample_kernel(RoundArgs a, uint32_t round) {
    constexpr uint32_t kNoBlock = 0xFFFFFFFFu;   // start of the entries past the list
    if (a.picks && !a.all[round - 1]) return;   // the picks of section 6 draw this round
    if (kSingle && round <= kPreRounds && a.pre_list[round - 1]) {
        const uint32_t cnt = *a.pre_cnt[round - 1];
        if (cnt <= a.pre_cap) {   // uniform: the round's draws were taken ahead
            sample_from_list<K>(a, a.pre_list[round - 1], cnt);
            return;
        }
    }
    const uint32_t total = (uint32_t)a.ctr->blocks;
    const uint32_t nsl = a.ctr->n_slices;
    const K* B = (const K*)a.B;
    const uint4* sl = a.slices;
    const uint32_t lane = lane_id();
    const uint32_t W = gridDim.x * (kT / kWave);
    const uint32_t w = blockIdx.x * (kT / kWave) + threadIdx.x / kWave;
    const uint32_t b_lo = (uint32_t)((uint64_t)total * w / W);
    const uint32_t b_hi = (uint32_t)((uint64_t)total * (w + 1) / W);
    if (b_lo >= b_hi) return;   // uniform over the wave

    // slice of block b_lo: the last entry starting at or before it, by a
    // 64-way search (entry 0 starts at block 0)
    uint32_t lo = 0, hi = nsl;   // answer in [lo, hi)
    while (hi - lo > (uint32_t)kWave) {
        const uint32_t step = (hi - lo + kWave - 1) / kWave;
        const uint32_t q = lo + lane * step;
        const uint32_t c = (uint32_t)__popcll(__ballot(q < hi && sl[q].x <= b_lo));
        lo += (c - 1) * step;
        hi = min(lo + step, hi);
    }
    uint32_t jq = lo + (uint32_t)__popcll(__ballot(lo + lane < hi && sl[lo + lane].x <= b_lo)) - 1;

    // parameters of the lane's current interval (instance seed, rate, base);
    // the same for every lane when the engine holds one instance
    constexpr bool single = kSingle;
    uint32_t cur_k = kNoBlock, th = 0;
    bool take_all = false;
    uint64_t seed = 0, pos0 = 0;
    if (single) {
        seed = a.run[0].seed;
        pos0 = a.inst[0].pos0;
        th = a.thresh[round - 1];
        take_all = a.all[round - 1] != 0;
    }

    // per-wave staging of the emitted probes: one slot reservation per
    // kSampleStage probes instead of one per step (a single counter takes
    // every reservation of the round)
    __shared__ uint64_t stage_key[kT / kWave][kSampleStage];
    __shared__ uint32_t stage_tag[kT / kWave][kSampleStage];
    __shared__ uint32_t stage_ivl[kT / kWave][kSampleStage];
    uint64_t* st_key = stage_key[threadIdx.x / kWave];
    uint32_t* st_tag = stage_tag[threadIdx.x / kWave];
    uint32_t* st_ivl = stage_ivl[threadIdx.x / kWave];
    uint32_t fill = 0;

    uint4 e = jq + lane < nsl ? sl[jq + lane] : make_uint4(kNoBlock, 0, 0, 0);
    uint32_t nxt = jq + kWave < nsl ? sl[jq + kWave].x : kNoBlock;
    for (uint32_t b0 = b_lo; b0 < b_hi; b0 += kWave) {
        // the window of the next step, loaded while this one draws
        const uint32_t bn = b0 + kWave;
        const uint32_t jn = jq + (uint32_t)__popcll(__ballot(e.x <= bn)) + (nxt <= bn ? 1u : 0u) - 1;
        uint4 en = make_uint4(kNoBlock, 0, 0, 0);
        uint32_t nxtn = kNoBlock;
        if (bn < b_hi) {   // uniform
            if (jn + lane < nsl) en = sl[jn + lane];
            if (jn + kWave < nsl) nxtn = sl[jn + kWave].x;
        }
        // slice of this lane's block: the last window entry starting at or
        // before it (entry starts increase across the lanes)
        const uint32_t b = b0 + lane;
        uint32_t pos = 0;
        if (__builtin_amdgcn_readlane(e.x, 1) > b0 + (kWave - 1)) {
            pos = 0;   // the first slice holds the whole step
        } else {
#pragma unroll
            for (uint32_t st = kWave / 2; st > 0; st >>= 1)
                if ((uint32_t)__shfl(e.x, (int)(pos + st)) <= b) pos += st;
        }
        const uint32_t s_first = __shfl(e.x, (int)pos);
        const uint32_t ga = __shfl(e.y, (int)pos);
        const uint32_t gb = __shfl(e.z, (int)pos);
        const uint32_t k = __shfl(e.w, (int)pos);
        uint32_t hits = 0;   // bit q: tag 4 blk + q is a probe
        uint64_t blk = 0;
        if (b < b_hi) {
            if (!single && k != cur_k) {
                cur_k = k;
                const uint32_t I = a.ivl_inst[k];
                seed = a.run[I].seed;
                pos0 = a.inst[I].pos0;
                th = a.thresh[(uint64_t)I * a.J + (round - 1)];
                take_all = a.all[(uint64_t)I * a.J + (round - 1)] != 0;
            }
            // tags are below 2^32, so block and tag fit 32 bits
            const uint32_t blk32 = (ga >> 2) + (b - s_first);
            blk = blk32;
            const Philox4 r = sample_block(seed, blk, round);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (take_all || r.v[q] < th) hits |= 1u << q;
            // the first and last block of a slice may hold tags outside it
            const uint32_t g0 = blk32 * 4;
            if (g0 < ga || (uint64_t)g0 + 4 > gb) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (g0 + q < ga || g0 + q >= gb) hits &= ~(1u << q);
            }
        }
        if (__ballot(hits != 0)) {
            // the probes go to the wave's staging area in LDS (at most 4 per
            // lane, so one step always fits once the area is flushed)
            const uint32_t c = __popc(hits);
            const uint32_t inc = wave_inclusive_scan<uint32_t>(c);
            const uint32_t total = (uint32_t)__shfl((int)inc, kWave - 1);
            if (fill + total > kSampleStage) {
                flush_stage(a, st_key, st_tag, st_ivl, fill);
                fill = 0;
            }
            uint32_t o = fill + inc - c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (hits & (1u << q)) {
                    const uint32_t g = (uint32_t)(blk * 4 + q);
                    st_key[o] = (uint64_t)B[pos0 + g];
                    st_tag[o] = g;
                    st_ivl[o] = k;
                    ++o;
                }
            }
            fill += total;
        }
        e = en;
        nxt = nxtn;
        jq = jn;
    }
    if (fill) flush_stage(a, st_key, st_tag, st_ivl, fill);
}

// Section 6's sampler (one instance): thread per pick l of segment s, a
// uniform position of the segment from Philox word 0 of counter (l, s, j, 1),
// floor(word n_s / 2^32).  The pick is kept when it lies in the slice of an
// interval in its segment (one binary search, as above) and its tag's bit
// was not yet set this round (a position picked twice is one probe).
template <typename K>
__global__ __launch_bounds__(kT) void pick_sample_kernel(RoundArgs a, uint32_t round) {
    if (halted(a) || a.all[round - 1]) return;
    const uint32_t n_ivl = a.ctr->n_ivl;
    if (n_ivl == 0) return;
    const InstDesc D = a.inst[0];
    const uint32_t picks = a.thresh[round - 1];
    const uint64_t total = (uint64_t)D.p * picks;
    const uint64_t seed = a.run[0].seed;
    const K* B = (const K*)a.B;
    const uint32_t lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // whole waves step together (the probe slots are taken once per wave)
    for (uint64_t xb = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); xb < total; xb += stride) {
        const uint64_t x = xb + lane;
        bool take = x < total;
        uint32_t kl = 0;
        uint64_t g = 0;
        if (take) {
            const uint32_t s = (uint32_t)(x / picks), l = (uint32_t)(x - (uint64_t)s * picks);
            const uint32_t seg = D.seg0 + s;
            const uint64_t sb = a.seg_off[seg] - D.pos0;
            const uint64_t ns = a.seg_off[seg + 1] - a.seg_off[seg];
            const Philox4 w = philox10(l, s, round, 1u, (uint32_t)seed, (uint32_t)(seed >> 32));
            g = sb + (((uint64_t)w.v[0] * ns) >> 32);
            auto bounds = [&](uint32_t k, uint64_t* ga, uint64_t* gb) {
                const uint32_t row = a.ivl_row[k];
                slice_bounds(a, D, row - D.row0, s, a.lrank[row] == kNone, a.urank[row] == kNone, ga, gb);
            };
            uint32_t kh = n_ivl;   // the last interval whose slice starts at or before g
            uint64_t ga, gb;
            bounds(0, &ga, &gb);
            if (ga > g) {
                take = false;
            } else {
                while (kh - kl > 1) {
                    const uint32_t mid = (kl + kh) >> 1;
                    uint64_t ma, mb;
                    bounds(mid, &ma, &mb);
                    if (ma <= g) kl = mid; else kh = mid;
                }
                bounds(kl, &ga, &gb);
                take = g >= ga && g < gb;
            }
            if (take) {
                const uint32_t bit = 1u << (g & 31);
                take = (atomicOr(&a.pick_bits[(D.pos0 >> 5) + (g >> 5)], bit) & bit) == 0;
            }
        }
        const uint64_t mask = __ballot(take);
        if (!mask) continue;   // uniform
        unsigned long long base = 0;
        const int leader = __ffsll((long long)mask) - 1;
        if ((int)lane == leader) base = atomicAdd(&a.ctr->m, (unsigned long long)__popcll(mask));
        base = shfl_u64(base, leader);
        bool stored = false;
        if (take) {
            const uint64_t o = base + __popcll(mask & lanes_below_mask());
            if (o < a.cap) {
                a.pr_key[o] = (uint64_t)B[D.pos0 + g];
                a.pr_tag[o] = g;
                a.pr_ivl[o] = kl;
                stored = true;
            } else {
                atomicOr(&a.ctr->overflow, 1u);
            }
        }
        add_interval_counts(a.ivl_pcnt, kl, stored ? 1u : 0u);
    }
}

// The bits of this round's kept picks, cleared for the next round (every
// set bit belongs to a stored probe unless the probe buffers overran, when
// the whole map is cleared before the rounds start again).
__global__ void pick_clear_kernel(RoundArgs a) {
    const uint64_t m = min(a.ctr->m_stored, a.cap);
    const uint64_t pos0 = a.inst[0].pos0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        a.pick_bits[(pos0 >> 5) + (a.pr_tag[e] >> 5)] = 0;
}

__global__ void pick_clear_all_kernel(uint32_t* bits, uint64_t words) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        bits[i] = 0;
}

// Fixed probe budget (one instance): the round's acceptance threshold from
// the domain just measured, floor(q 2^32) with q = c p / |gamma| in double,
// or every tag when q >= 1.
__global__ void budget_rate_kernel(RoundArgs a, uint32_t round) {
    if (halted(a)) return;
    const uint32_t n_ivl = a.ctr->n_ivl;
    // thread per instance: its intervals are a contiguous run of the list (the
    // leaders are found in row order, and rows in instance order)
    for (uint32_t I = blockIdx.x * blockDim.x + threadIdx.x; I < a.n_inst; I += gridDim.x * blockDim.x) {
        // [k0, k1): the intervals of instance I; ivl_dom holds the domain
        // before every interval
        auto first_of = [&](uint32_t inst) {
            uint32_t lo = 0, hi = n_ivl;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (a.ivl_inst[mid] < inst) lo = mid + 1; else hi = mid;
            }
            return lo;
        };
        const uint32_t k0 = first_of(I), k1 = first_of(I + 1);
        const uint64_t dom = a.ivl_dom[k1] - a.ivl_dom[k0];
        if (dom == 0) continue;   // no interval left in this instance
        const InstDesc& D = a.inst[I];
        bool all;
        uint32_t th;
        if (a.picks) {
            // section 6: ceil(c N / |gamma|) picks of every segment, or every
            // key of the intervals once that reaches the largest segment
            const double d = ceil(((double)a.budget * (double)D.n) / (double)dom);
            const uint64_t max_seg = (D.n + D.p - 1) / D.p;
            all = d >= (double)max_seg;
            th = all ? 0xFFFFFFFFu : (uint32_t)d;
        } else {
            const double q = ((double)a.budget * (double)D.q) / (double)dom;
            all = q >= 1.0;
            th = all ? 0xFFFFFFFFu : (uint32_t)floor(q * 4294967296.0);
        }
        a.thresh[(uint64_t)I * a.J + round - 1] = th;
        a.all[(uint64_t)I * a.J + round - 1] = all ? 1 : 0;
    }
}

// One workgroup: where every interval's probes go in sorted order, how many
// ordering workgroups it takes, every instance's probe range and count-matrix
// block; flags a capacity overrun.
template <int kScanT>
__global__ __launch_bounds__(kScanT) void probe_scan_kernel(RoundArgs a, uint32_t round) {
    __shared__ uint64_t scratch[kScanT / kWave];
    RoundCounters* c = a.ctr;
    const uint64_t m = c->m;
    // the sampler may already have flagged an overrun: record how many probes
    // the round needs before anything else
    if (threadIdx.x == 0 && m > c->m_max) c->m_max = m;
    if (halted(a)) return;
    if (threadIdx.x == 0) {
        a.hist[round - 1].domain = c->domain;
        a.hist[round - 1].m = m;
        a.hist[round - 1].thresh = a.thresh[round - 1];
        a.hist[round - 1].all = a.all[round - 1];
    }
    if (m > a.cap) {
        if (threadIdx.x == 0) c->overflow = 1u;
        return;
    }
    const uint32_t n = c->n_ivl;
    const uint32_t per = (n + kScanT - 1) / kScanT;
    const uint32_t r0 = min(threadIdx.x * per, n), r1 = min(r0 + per, n);
    uint64_t lp = 0, lt = 0;
    for (uint32_t k = r0; k < r1; ++k) {
        const uint32_t pc = a.ivl_pcnt[k];
        lp += pc;
        lt += (pc + kOrderLanes - 1) / kOrderLanes;
    }
    uint64_t tp, tt;
    uint64_t rp = block_exclusive_scan<uint64_t, kScanT>(lp, scratch, &tp);
    uint64_t rt = block_exclusive_scan<uint64_t, kScanT>(lt, scratch, &tt);
    for (uint32_t I = threadIdx.x; I < a.n_inst; I += kScanT) {
        a.inst_plo[I] = 0;
        a.inst_pm[I] = 0;
    }
    __syncthreads();
    for (uint32_t k = r0; k < r1; ++k) {
        const uint32_t pc = a.ivl_pcnt[k];
        const uint32_t I = a.ivl_inst[k];
        a.ivl_poff[k] = (uint32_t)rp;
        a.ivl_tile0[k] = (uint32_t)rt;
        if (k == 0 || a.ivl_inst[k - 1] != I) a.inst_plo[I] = (uint32_t)rp;
        if (k + 1 == n || a.ivl_inst[k + 1] != I) a.inst_pm[I] = (uint32_t)(rp + pc);   // end, for now
        rp += pc;
        rt += (pc + kOrderLanes - 1) / kOrderLanes;
    }
    __syncthreads();
    // probe counts and count-matrix blocks of the instances
    const uint32_t ni = a.n_inst;
    const uint32_t pi = (ni + kScanT - 1) / kScanT;
    const uint32_t i0 = min(threadIdx.x * pi, ni), i1 = min(i0 + pi, ni);
    uint64_t lc = 0;
    for (uint32_t I = i0; I < i1; ++I) {
        const uint32_t end = a.inst_pm[I];
        const uint32_t mI = end ? end - a.inst_plo[I] : 0u;
        lc += (uint64_t)mI * a.inst[I].p;
    }
    uint64_t tc;
    uint64_t rc = block_exclusive_scan<uint64_t, kScanT>(lc, scratch, &tc);
    for (uint32_t I = i0; I < i1; ++I) {
        const uint32_t end = a.inst_pm[I];
        const uint32_t mI = end ? end - a.inst_plo[I] : 0u;
        a.inst_pm[I] = mI;
        a.cm_off[I] = rc;
        rc += (uint64_t)mI * a.inst[I].p;
    }
    if (threadIdx.x == 0) {
        a.ivl_poff[n] = (uint32_t)tp;
        a.ivl_tile0[n] = (uint32_t)tt;
        c->m_stored = tp;
        c->tiles = (uint32_t)tt;
        c->cm_need = tc;
        if (tc > c->cm_max) c->cm_max = tc;
        if (tc > a.cm_cap || tp != m) c->overflow = 1u;
    }
}

// Thread per emitted probe: into its interval's range (any order inside).
// A wave whose probes all belong to one interval takes its slots with one
// atomic; otherwise every probe takes its own.
__global__ void group_kernel(RoundArgs a) {
    if (halted(a)) return;
    const uint64_t m = a.ctr->m_stored;
    const uint32_t lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; o0 < m; o0 += stride) {
        const uint64_t o = o0 + lane;
        const bool valid = o < m;
        const uint32_t k = valid ? a.pr_ivl[o] : 0u;
        uint32_t slot = 0;
        const uint64_t live = __ballot(valid);
        const uint32_t k0 = __shfl(k, __ffsll((unsigned long long)live) - 1);
        if (__ballot(valid && k != k0) == 0) {
            // one interval for the whole wave (round 1 has a single one): one atomic
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&a.ivl_cursor[k0], (uint32_t)__popcll(live));
            base = __shfl(base, 0);
            slot = base + (uint32_t)__popcll(live & lanes_below_mask());
        } else if (valid) {
            slot = atomicAdd(&a.ivl_cursor[k], 1u);
        }
        if (valid) {
            const uint64_t gi = (uint64_t)a.ivl_poff[k] + slot;
            a.g_key[gi] = a.pr_key[o];
            a.g_tag[gi] = a.pr_tag[o];
        }
    }
}

// The splitter row of interval k with its open-end flags, kept with each
// sorted probe so that the rank search reads it with the probe.
__device__ __forceinline__ uint32_t probe_row(const RoundArgs& a, uint32_t k) {
    const uint32_t row = a.ivl_row[k];
    return row | (a.lrank[row] == kNone ? kRowLNone : 0u) | (a.urank[row] == kNone ? kRowUNone : 0u);
}

// Tile of kOrderLanes probes of one interval: each probe's place among the
// interval's probes in the order (key, tag), counted by 32 lanes of a wave
// (every 32nd probe of the interval each) against chunks of the interval
// staged in LDS; the probe goes to that place of the sorted arrays, with its
// segment, and its rank sum is cleared.  Workgroups stride over the tiles.
__global__ __launch_bounds__(kOrderThreads) void order_kernel(RoundArgs a) {
    constexpr uint32_t kTile = 1024;
    constexpr uint32_t kParts = kOrderThreads / kOrderLanes;
    static_assert(kParts == kWave / 2, "a probe's parts are half a wave");
    __shared__ uint64_t tk[kTile];
    __shared__ uint64_t tt[kTile];
    if (halted(a)) return;
    const uint32_t tiles = a.ctr->tiles;
    const uint32_t n_ivl = a.ctr->n_ivl;
    const uint32_t part = threadIdx.x % kParts, pl = threadIdx.x / kParts;
    for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {   // uniform
        const uint32_t k = last_le(a.ivl_tile0, n_ivl, t);
        const uint32_t base = a.ivl_poff[k];
        const uint32_t nk = a.ivl_poff[k + 1] - base;
        const uint32_t i = (t - a.ivl_tile0[k]) * kOrderLanes + pl;
        const bool valid = i < nk;
        const uint64_t key = valid ? a.g_key[base + i] : 0;
        const uint64_t tag = valid ? a.g_tag[base + i] : 0;
        uint32_t c = 0;
        for (uint32_t c0 = 0; c0 < nk; c0 += kTile) {
            const uint32_t nc = min(kTile, nk - c0);
            __syncthreads();   // the previous chunk is no longer read
            for (uint32_t x = threadIdx.x; x < nc; x += kOrderThreads) {
                tk[x] = a.g_key[base + c0 + x];
                tt[x] = a.g_tag[base + c0 + x];
            }
            __syncthreads();
#pragma unroll 4
            for (uint32_t j = part; j < nc; j += kParts) {
                const uint64_t kj = tk[j], tj = tt[j];
                c += (kj < key || (kj == key && tj < tag)) ? 1u : 0u;
            }
        }
#pragma unroll
        for (uint32_t off = kParts / 2; off > 0; off >>= 1) c += (uint32_t)__shfl_xor((int)c, (int)off);
        if (part == 0 && valid) {
            const uint64_t pos = base + c;
            const InstDesc& D = a.inst[a.ivl_inst[k]];
            // segment of the probe: the last segment of the instance starting at or before it
            uint32_t lo = 0, hi = D.p;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (a.seg_off[D.seg0 + mid] - D.pos0 <= tag) lo = mid; else hi = mid;
            }
            a.ps_key[pos] = key;
            a.ps_tag[pos] = tag;
            a.ps_ivl[pos] = k;
            a.ps_seg[pos] = D.seg0 + lo;
            a.ps_row[pos] = probe_row(a, k);
            a.pr_rank[pos] = 0;   // the rank reduction adds into it
        }
    }
}

// (key_e, g_e) after (kx, gx) in the order (key, tag)?
__device__ __forceinline__ bool after(uint64_t ke, uint64_t ge, uint64_t kx, uint64_t gx) {
    return ke > kx || (ke == kx && ge > gx);
}

// Workgroup per (segment s, chunk of kRankChunk keys): the probes of the
// segment's instance whose count c_s(e) falls in the chunk are the sorted run
// [e0, e1); each finds its place among the chunk's fences in LDS, then inside
// one kFenceStride-key block of B.  c_s(e) goes to the instance's count matrix
// (segment-major).
template <typename K>
__global__ __launch_bounds__(256) void rank_kernel(RoundArgs a) {
    __shared__ uint64_t F[kRankFences];
    __shared__ uint32_t sh_e[2];
    __shared__ uint32_t sh_cnt[2];
    const uint32_t c = blockIdx.x;
    if (c >= a.n_chunks || halted(a)) return;
    const uint32_t s = a.chunk_seg[c];
    const uint32_t I = a.seg_inst[s];
    const uint32_t m = a.inst_pm[I];
    if (m == 0) return;
    const uint32_t plo = a.inst_plo[I];
    const InstDesc& D = a.inst[I];
    const uint32_t s_local = s - D.seg0;
    const uint64_t sb = a.seg_off[s];
    const uint64_t ns = a.seg_off[s + 1] - sb;
    const uint64_t g_sb = sb - D.pos0;   // tag of the segment's first key
    const uint64_t lo_pos = a.chunk_lo[c];
    const uint64_t chunk_end = min(lo_pos + kRankChunk, ns);
    const bool last = chunk_end == ns;
    const K* B = (const K*)a.B + sb;
    const uint64_t* pk = a.ps_key + plo;
    const uint64_t* pt = a.ps_tag + plo;
    // [e0, e1): the probes with c_s(e) in the chunk.  The first probe with
    // c_s(e) >= x (x >= 1) is the first probe after the element at position
    // x - 1 of the segment.  Two parallel steps: 256 evenly spaced probes
    // bracket the answer, then every probe of the bracket is tested.
    const bool need0 = lo_pos != 0, need1 = !last;
    // no probe after the boundary element: m; no boundary (first chunk): 0
    if (threadIdx.x < 2) sh_e[threadIdx.x] = (threadIdx.x == 0 && !need0) ? 0 : m;
    if (threadIdx.x == 0) sh_cnt[0] = sh_cnt[1] = 0;
    __syncthreads();
    const uint32_t step = (m + 255) / 256;
    uint64_t bx[2], bg[2];
    bx[0] = need0 ? (uint64_t)B[lo_pos - 1] : 0;
    bg[0] = g_sb + lo_pos - 1;
    bx[1] = need1 ? (uint64_t)B[chunk_end - 1] : 0;
    bg[1] = g_sb + chunk_end - 1;
    {
        const uint64_t j = (uint64_t)threadIdx.x * step;
        if (j < m) {
            const uint64_t kj = pk[j], gj = pt[j];
            if (need0 && !after(kj, gj, bx[0], bg[0])) atomicAdd(&sh_cnt[0], 1u);
            if (need1 && !after(kj, gj, bx[1], bg[1])) atomicAdd(&sh_cnt[1], 1u);
        }
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
        if (!(q == 0 ? need0 : need1)) continue;   // uniform
        // cn samples are not after the boundary (the predicate is monotone over
        // the sorted probes), so the answer lies in [(cn-1)*step + 1, cn*step],
        // or is m when no probe of that range is after it
        const uint32_t cn = sh_cnt[q];
        const uint32_t lo = cn == 0 ? 0 : (cn - 1) * step + 1;
        const uint32_t hi = (uint32_t)min((uint64_t)cn * step + 1, (uint64_t)m);   // exclusive
        for (uint32_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            if (after(pk[e], pt[e], bx[q], bg[q]) && (e == 0 || !after(pk[e - 1], pt[e - 1], bx[q], bg[q])))
                sh_e[q] = e;   // exactly one e qualifies
        }
    }
    __syncthreads();
    const uint32_t e0 = sh_e[0], e1 = sh_e[1];
    if (e0 >= e1) return;   // no probe counts into this chunk (uniform over the workgroup)
    const uint32_t nf = (uint32_t)((chunk_end - lo_pos + kFenceStride - 1) / kFenceStride);
    const uint64_t* fsrc = a.fences.key + a.fences.base[s] + lo_pos / kFenceStride;
    for (uint32_t i = threadIdx.x; i < nf; i += blockDim.x) F[i] = fsrc[i];
    __syncthreads();
    uint32_t* out = a.cmat + a.cm_off[I] + (uint64_t)s_local * m;
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const K key = (K)pk[e];
        const uint64_t g = pt[e];
        const uint32_t t = a.ps_seg[plo + e];
        uint64_t cnt;
        if (t == s) {
            cnt = g - g_sb;
        } else {
            // equal keys of earlier segments precede the probe, of later ones follow
            const bool eqb = s < t;
            uint32_t f0 = 0, f1 = nf;   // first fence that does not precede the probe
            while (f0 < f1) {
                const uint32_t mid = (f0 + f1) >> 1;
                const K x = (K)F[mid];
                if (eqb ? (x <= key) : (x < key)) f0 = mid + 1; else f1 = mid;
            }
            if (f0 == 0) {
                cnt = lo_pos;
            } else {
                const uint64_t lo = lo_pos + (uint64_t)(f0 - 1) * kFenceStride + 1;
                const uint64_t hi = f0 < nf ? lo_pos + (uint64_t)f0 * kFenceStride : chunk_end;
                cnt = count_before<K>(B, lo, hi, key, eqb);
            }
        }
        out[e] = (uint32_t)cnt;
    }
}

// First probe of [lo, hi) (sorted by (key, tag)) after the element (bx, bg),
// hi when none is; all 256 threads of the workgroup call it.  Two parallel
// steps: 256 evenly spaced probes bracket the answer, then every probe of
// the bracket is tested (the predicate is monotone over the sorted probes).
__device__ uint32_t first_after(const uint64_t* pk, const uint64_t* pt, uint32_t lo, uint32_t hi,
                                uint64_t bx, uint64_t bg, uint32_t* sh_cnt, uint32_t* sh_e) {
    __syncthreads();
    if (threadIdx.x == 0) {
        *sh_cnt = 0;
        *sh_e = hi;
    }
    __syncthreads();
    const uint32_t n = hi - lo;
    const uint32_t step = (n + 255) / 256;
    {
        const uint64_t j = lo + (uint64_t)threadIdx.x * step;
        if (j < hi && !after(pk[j], pt[j], bx, bg)) atomicAdd(sh_cnt, 1u);
    }
    __syncthreads();
    const uint32_t cn = *sh_cnt;
    const uint32_t a0 = cn == 0 ? lo : lo + (cn - 1) * step + 1;
    const uint32_t a1 = (uint32_t)min((uint64_t)lo + (uint64_t)cn * step + 1, (uint64_t)hi);
    for (uint32_t e = a0 + threadIdx.x; e < a1; e += blockDim.x)
        if (after(pk[e], pt[e], bx, bg) && (e == lo || !after(pk[e - 1], pt[e - 1], bx, bg))) *sh_e = e;
    __syncthreads();
    return *sh_e;
}

// Round 1 with probes denser than the fences (one-round HSS, full samples):
// workgroup per (segment s, chunk of kRankChunk keys) as rank_kernel, but the
// chunk's keys are staged in LDS tile by tile and every probe whose count
// falls in a tile is placed by binary search in the tile -- no read of B per
// (probe, segment).
template <typename K>
__global__ __launch_bounds__(256) void rank_dense_kernel(RoundArgs a) {
    __shared__ K T[kDenseTile];
    __shared__ uint32_t sh_cnt, sh_e;
    const uint32_t c = blockIdx.x;
    if (c >= a.n_chunks || halted(a)) return;
    const uint32_t s = a.chunk_seg[c];
    const uint32_t I = a.seg_inst[s];
    const uint32_t m = a.inst_pm[I];
    if (m == 0) return;
    const uint32_t plo = a.inst_plo[I];
    const InstDesc& D = a.inst[I];
    const uint32_t s_local = s - D.seg0;
    const uint64_t sb = a.seg_off[s];
    const uint64_t ns = a.seg_off[s + 1] - sb;
    const uint64_t g_sb = sb - D.pos0;
    const uint64_t lo_pos = a.chunk_lo[c];
    const uint64_t chunk_end = min(lo_pos + kRankChunk, ns);
    const K* B = (const K*)a.B + sb;
    const uint64_t* pk = a.ps_key + plo;
    const uint64_t* pt = a.ps_tag + plo;
    uint32_t* out = a.cmat + a.cm_off[I] + (uint64_t)s_local * m;
    // probes with c_s(e) >= x: from the first probe after element x - 1
    uint32_t ea = lo_pos == 0 ? 0 : first_after(pk, pt, 0, m, (uint64_t)B[lo_pos - 1], g_sb + lo_pos - 1,
                                                &sh_cnt, &sh_e);
    for (uint64_t ta = lo_pos; ta < chunk_end; ta += kDenseTile) {
        const uint64_t tb = min(ta + (uint64_t)kDenseTile, chunk_end);
        // [ea, eb): the probes with c_s(e) in [ta, tb) (the segment's last
        // tile also takes the probes after all its keys)
        const uint32_t eb = tb == ns ? m
                                     : first_after(pk, pt, ea, m, (uint64_t)B[tb - 1], g_sb + tb - 1,
                                                   &sh_cnt, &sh_e);
        if (ea < eb) {   // uniform over the workgroup
            __syncthreads();
            const uint32_t nt = (uint32_t)(tb - ta);
            for (uint32_t i = threadIdx.x; i < nt; i += blockDim.x) T[i] = B[ta + i];
            __syncthreads();
            for (uint32_t e = ea + threadIdx.x; e < eb; e += blockDim.x) {
                // keys below the probe's key: its count unless the tile holds
                // its key (then the tie rule of the order (key, tag) decides)
                const K key = (K)pk[e];
                uint32_t lo = 0, hi = nt;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (T[mid] < key) lo = mid + 1; else hi = mid;
                }
                uint64_t cnt = ta + lo;
                if (lo < nt && T[lo] == key) {
                    const uint32_t t = a.ps_seg[plo + e];
                    if (t == s) {
                        cnt = pt[e] - g_sb;
                    } else if (s < t) {
                        // equal keys of earlier segments precede the probe
                        uint32_t l2 = lo, h2 = nt;
                        while (l2 < h2) {
                            const uint32_t mid = (l2 + h2) >> 1;
                            if (T[mid] <= key) l2 = mid + 1; else h2 = mid;
                        }
                        cnt = ta + l2;
                    }
                }
                out[e] = (uint32_t)cnt;
            }
        }
        ea = eb;
    }
}

// Rounds after the first: probe e lies strictly inside its interval, so its
// count in segment s lies in the interval's slice [lo, hi) of s (section
// 4.2.2: the search is confined to the splitter interval).  An empty slice
// gives lo without a read; a short one is searched directly; a longer one
// through its own fences first, then one kFenceStride-key block.  Thread per
// (probe, segment) pair, in count-matrix order (probes of one segment on
// consecutive threads).
template <typename K>
__global__ __launch_bounds__(256) void rank_pairs_kernel(RoundArgs a) {
    if (halted(a)) return;
    const uint64_t total = a.ctr->cm_need;
    const K* B = (const K*)a.B;
    for (uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * 256) {
        const uint32_t I = a.n_inst > 1 ? last_le(a.cm_off, a.n_inst, x) : 0u;
        const uint32_t m = a.inst_pm[I];
        const uint64_t rem = x - a.cm_off[I];
        const uint32_t sl = (uint32_t)(rem / m);
        const uint64_t e = a.inst_plo[I] + rem % m;
        const InstDesc& D = a.inst[I];
        const uint32_t s = D.seg0 + sl;
        const uint64_t s0 = a.seg_off[s];              // position of the segment
        const uint32_t t = a.ps_seg[e];
        uint64_t cnt;
        if (t == s) {
            cnt = a.ps_tag[e] - (s0 - D.pos0);         // its own place
        } else {
            const uint32_t rf = a.ps_row[e];
            const uint32_t row = rf & kRowMask;
            const uint64_t cell = D.tab0 + (uint64_t)(row - D.row0) * D.p + sl;
            const uint64_t lo = (rf & kRowLNone) ? 0 : a.lpos[cell];
            const uint64_t hi = (rf & kRowUNone) ? a.seg_off[s + 1] - s0 : a.upos[cell];
            if (hi <= lo) {
                cnt = lo;
            } else {
                const K key = (K)a.ps_key[e];
                const bool eqb = s < t;   // equal keys of earlier segments precede
                const K* Bs = B + s0;
                uint64_t q0 = lo, q1 = hi;
                if (hi - lo > 2 * kFenceStride) {
                    // fences f with f * kFenceStride in [lo, hi): the counted
                    // ones form a prefix; the answer follows the last of them
                    const uint64_t* F = a.fences.key + a.fences.base[s];
                    uint64_t f0 = (lo + kFenceStride - 1) / kFenceStride;
                    const uint64_t fl = f0;
                    uint64_t f1 = (hi + kFenceStride - 1) / kFenceStride;
                    const uint64_t fh = f1;
                    while (f0 < f1) {
                        const uint64_t mid = (f0 + f1) >> 1;
                        const K fk = (K)F[mid];
                        if (eqb ? (fk <= key) : (fk < key)) f0 = mid + 1; else f1 = mid;
                    }
                    if (f0 > fl) q0 = (f0 - 1) * kFenceStride + 1;
                    if (f0 < fh) q1 = f0 * kFenceStride;
                }
                cnt = count_before<K>(Bs, q0, q1, key, eqb);
            }
        }
        a.cmat[x] = (uint32_t)cnt;
    }
}

// Sorted-probe path (large rounds sorted by the segmented sort): the
// interval offsets as 64-bit segment bounds for the sort.
__global__ void probe_offsets_kernel(RoundArgs a, uint64_t* __restrict__ out) {
    const uint32_t n = a.ctr->n_ivl;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= n; k += gridDim.x * blockDim.x)
        out[k] = a.ivl_poff[k];
}

// Sorted-probe path: the probes are in (key, tag) order inside their
// interval's range; each gets its interval, its segment and a cleared rank
// sum, as the ordering kernel would give them.
__global__ void probe_finish_kernel(RoundArgs a) {
    if (halted(a)) return;
    const uint64_t m = a.ctr->m_stored;
    const uint32_t n_ivl = a.ctr->n_ivl;
    for (uint64_t pos = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < m;
         pos += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = last_le(a.ivl_poff, n_ivl, (uint32_t)pos);
        const InstDesc& D = a.inst[a.ivl_inst[k]];
        const uint64_t tag = a.ps_tag[pos];
        uint32_t lo = 0, hi = D.p;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.seg_off[D.seg0 + mid] - D.pos0 <= tag) lo = mid; else hi = mid;
        }
        a.ps_ivl[pos] = k;
        a.ps_seg[pos] = D.seg0 + lo;
        a.ps_row[pos] = probe_row(a, k);
        a.pr_rank[pos] = 0;
    }
}

// The reduction of section 5.2: R(e) is the sum over the instance's segments
// of c_s(e), the column sums of its count matrix.  Tiles of 256 sorted probes
// x kReduceRows segments; the partial sums are integers, so the order of the
// atomic additions does not change R(e).
__global__ __launch_bounds__(256) void reduce_kernel(RoundArgs a) {
    if (halted(a)) return;
    const uint64_t m_all = a.ctr->m_stored;
    const uint64_t etiles = (m_all + 255) / 256;
    const uint64_t tiles = etiles * ((a.p_max + kReduceRows - 1) / kReduceRows);
    // consecutive workgroups take consecutive probe tiles of one segment group
    for (uint64_t x = blockIdx.x; x < tiles; x += gridDim.x) {
        const uint64_t e = (x % etiles) * 256 + threadIdx.x;
        const uint32_t s0 = (uint32_t)(x / etiles) * kReduceRows;
        if (e >= m_all) continue;
        const uint32_t I = a.ivl_inst[a.ps_ivl[e]];
        const uint32_t p = a.inst[I].p;
        if (s0 >= p) continue;
        const uint32_t s1 = min(s0 + kReduceRows, p);
        const uint32_t m = a.inst_pm[I];
        const uint32_t* col = a.cmat + a.cm_off[I] + (e - a.inst_plo[I]);
        uint64_t sum = 0;
#pragma unroll
        for (uint32_t q = 0; q < kReduceRows; ++q)
            if (s0 + q < s1) sum += col[(uint64_t)(s0 + q) * m];
        atomicAdd((unsigned long long*)&a.pr_rank[e], (unsigned long long)sum);
    }
}

// Workgroup per splitter row (section 4.2.2 steps 3 and 5).  A probe whose
// rank lies in the target range settles the splitter (closest to N i/p, the
// lower rank on a tie); otherwise L and U move to the closest probe ranks
// below and above N i/p.  Every new bound or splitter probe is put in the
// row's two selection slots; its per-segment counts (its column of the count
// matrix) become row i of lpos (L), upos (U) or prow (the splitter) in
// settle_copy_kernel.  The grid also checks that ranks increase along every
// instance's sorted probes.
template <int kThreads>
__global__ __launch_bounds__(kThreads) void settle_kernel(RoundArgs a) {
    __shared__ uint32_t sh_cnt, sh_first;
    if (halted(a)) return;
    const uint64_t m_all = a.ctr->m_stored;
    for (uint64_t e = (uint64_t)blockIdx.x * kThreads + threadIdx.x; e + 1 < m_all;
         e += (uint64_t)gridDim.x * kThreads)
        if (a.ivl_inst[a.ps_ivl[e]] == a.ivl_inst[a.ps_ivl[e + 1]] && a.pr_rank[e] >= a.pr_rank[e + 1])
            atomicOr(&a.ctr->err, kErrRankOrder);
    const uint32_t r = blockIdx.x;
    if (r >= a.n_rows) return;
    if (a.settled[r]) {   // uniform over the workgroup: nothing to copy for this row
        if (threadIdx.x == 0) a.sel_e[2 * r] = a.sel_e[2 * r + 1] = kNoSel;
        return;
    }
    const uint32_t I = a.row_inst[r];
    const uint32_t mI = a.inst_pm[I];
    const uint64_t plo = a.inst_plo[I];
    const uint64_t* R = a.pr_rank + plo;
    const uint64_t target = a.ideal[r];
    // first probe with R >= N i / p, in two parallel steps: kThreads evenly
    // spaced probes bracket it, then every probe of the bracket is tested
    if (threadIdx.x == 0) { sh_cnt = 0; sh_first = mI; }
    __syncthreads();
    const uint32_t step = (mI + kThreads - 1) / kThreads;
    {
        const uint64_t j = (uint64_t)threadIdx.x * step;
        if (j < mI && R[j] < target) atomicAdd(&sh_cnt, 1u);
    }
    __syncthreads();
    {
        const uint32_t cn = sh_cnt;   // samples below the target
        const uint32_t blo = cn == 0 ? 0 : (cn - 1) * step + 1;
        const uint32_t bhi = (uint32_t)min((uint64_t)cn * step + 1, (uint64_t)mI);
        for (uint32_t e = blo + threadIdx.x; e < bhi; e += kThreads)
            if (R[e] >= target && (e == 0 || R[e - 1] < target)) sh_first = e;   // one e qualifies
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t sel0 = kNoSel, sel1 = kNoSel;
    uint8_t kind0 = 0;
    if (mI == 0) {   // no probe of this instance this round
        atomicAdd(&a.ctr->n_after, 1u);
    } else {
        const uint64_t tol = a.inst[I].tol;
        const uint64_t lo = sh_first;
        const bool has_above = lo < mI;
        const bool has_below = lo > 0;
        const uint64_t r_above = has_above ? R[lo] : 0;
        const uint64_t r_below = has_below ? R[lo - 1] : 0;
        const uint64_t d_above = r_above - target;
        const uint64_t d_below = target - r_below;
        int64_t pick = -1;
        if (has_below && d_below <= tol) pick = (int64_t)lo - 1;
        if (has_above && d_above <= tol && (pick < 0 || d_above < d_below)) pick = (int64_t)lo;
        if (pick >= 0) {
            const uint64_t e = plo + (uint64_t)pick;
            a.settled[r] = 1;
            a.chi[r] = R[pick];
            a.s_key[r] = a.ps_key[e];
            a.s_tag[r] = a.ps_tag[e];
            sel0 = (uint32_t)e;
            kind0 = 2;
        } else {
            atomicAdd(&a.ctr->n_after, 1u);
            if (has_below && (a.lrank[r] == kNone || r_below > a.lrank[r])) {
                a.lrank[r] = r_below;
                sel0 = (uint32_t)(plo + lo - 1);
                a.l_tag[r] = a.ps_tag[sel0];
            }
            if (has_above && r_above < a.urank[r]) {
                a.urank[r] = r_above;
                sel1 = (uint32_t)(plo + lo);
                a.u_tag[r] = a.ps_tag[sel1];
            }
        }
    }
    a.sel_e[2 * r] = sel0;
    a.sel_kind[2 * r] = kind0;
    a.sel_e[2 * r + 1] = sel1;
    a.sel_kind[2 * r + 1] = 1;
}

// The selected probes' per-segment counts into their table rows: workgroup
// per tile of kCopySlots consecutive selection slots x kCopySegs segments.
// The slots of consecutive rows select nearby sorted probes, so the tile's
// reads of one count-matrix row (segment) are nearly consecutive words; the
// tile is turned around in LDS and every slot's table row is written as
// kCopySegs consecutive words.  A lower bound's own segment gets +1 (its
// slice starts after the probe).
constexpr uint32_t kCopySlots = 64;
constexpr uint32_t kCopySegs = 32;

__global__ __launch_bounds__(256) void settle_copy_kernel(RoundArgs a) {
    __shared__ uint32_t T[kCopySegs][kCopySlots + 1];
    __shared__ uint32_t* dst_row[kCopySlots];
    __shared__ uint32_t own_seg[kCopySlots];
    __shared__ uint32_t seg_n[kCopySlots];
    if (halted(a)) return;
    const uint32_t n_slots = 2 * a.n_rows;
    const uint32_t slot_tiles = (n_slots + kCopySlots - 1) / kCopySlots;
    const uint32_t seg_tiles = (a.p_max + kCopySegs - 1) / kCopySegs;
    const uint32_t lane = lane_id(), w = threadIdx.x / kWave;
    for (uint64_t tile = blockIdx.x; tile < (uint64_t)slot_tiles * seg_tiles; tile += gridDim.x) {   // uniform
        const uint32_t stile = (uint32_t)(tile % slot_tiles), gtile = (uint32_t)(tile / slot_tiles);
        const uint32_t s0 = gtile * kCopySegs;
        // wave 0: the tile's slots (lane = slot)
        uint32_t e = kNoSel, I = 0, m = 0, sl_base = 0;
        uint64_t cm = 0;
        int has = 0;
        if (w == 0) {
            const uint32_t slot = stile * kCopySlots + lane;
            dst_row[lane] = nullptr;
            seg_n[lane] = 0;
            if (slot < n_slots) {
                e = a.sel_e[slot];
                if (e != kNoSel) {
                    const uint32_t r = slot / 2;
                    I = a.row_inst[r];
                    const InstDesc& D = a.inst[I];
                    if (s0 < D.p) {
                        const uint8_t kind = a.sel_kind[slot];
                        uint32_t* base = kind == 0 ? a.lpos : (kind == 1 ? a.upos : a.prow);
                        dst_row[lane] = base + D.tab0 + (uint64_t)(r - D.row0) * D.p;
                        own_seg[lane] = kind == 0 ? a.ps_seg[e] - D.seg0 : 0xFFFFFFFFu;
                        seg_n[lane] = min(D.p - s0, kCopySegs);
                        has = 1;
                    }
                }
            }
        }
        // a barrier that also tells whether any slot of the tile selects a
        // probe in these segments (uniform)
        if (!__syncthreads_or(has)) continue;
        // loads: wave w reads segments s0 + w, s0 + w + 4, ...; lane = slot
        {
            const uint32_t slot = stile * kCopySlots + lane;
            e = slot < n_slots ? a.sel_e[slot] : kNoSel;
            const uint32_t nseg = seg_n[lane];
            if (e != kNoSel && nseg) {
                I = a.row_inst[slot / 2];
                m = a.inst_pm[I];
                cm = a.cm_off[I];
                sl_base = e - a.inst_plo[I];
            }
            for (uint32_t q = w; q < kCopySegs; q += 256 / kWave) {
                uint32_t v = 0;
                if (e != kNoSel && q < nseg) v = a.cmat[cm + (uint64_t)(s0 + q) * m + sl_base];
                T[q][lane] = v;
            }
        }
        __syncthreads();
        // stores: kCopySegs consecutive words per slot
        for (uint32_t x = threadIdx.x; x < kCopySlots * kCopySegs; x += 256) {
            const uint32_t j = x / kCopySegs, q = x % kCopySegs;
            uint32_t* row = dst_row[j];
            if (row && q < seg_n[j]) row[s0 + q] = T[q][j] + (s0 + q == own_seg[j] ? 1u : 0u);
        }
        __syncthreads();   // the tile's LDS is rewritten by the next tile
    }
}

__global__ void finalize_kernel(RoundArgs a, uint64_t* chi_all) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < a.n_rows; r += gridDim.x * blockDim.x) {
        const uint32_t I = a.row_inst[r];
        const InstDesc& D = a.inst[I];
        const uint32_t i = r - D.row0;
        const uint64_t v = i == 0 ? 0 : (i == D.q ? D.n : a.chi[r]);
        chi_all[r] = v;
        a.run[I].offsets[i] = v;
    }
}

__global__ void segment_sources_kernel(RoundArgs a, const uint32_t* list, uint32_t count,
                                       uint64_t* key_src, uint64_t* val_src, int key_bytes) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < count; x += gridDim.x * blockDim.x) {
        const uint32_t s = list ? list[x] : x;
        const uint32_t I = a.seg_inst[s];
        const uint64_t rel = a.seg_off[s] - a.inst[I].pos0;
        key_src[x] = (uint64_t)(uintptr_t)a.run[I].kin + rel * (uint64_t)key_bytes;
        if (val_src) val_src[x] = a.run[I].vin ? (uint64_t)(uintptr_t)a.run[I].vin + rel * 8 : 0;
    }
}

__global__ void set_run_kernel(InstRun r, InstRun* dst) { *dst = r; }

unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 1u << 20) {
    const uint64_t g = (n + threads - 1) / threads;
    return (unsigned)(g == 0 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_counters_reset(RoundCounters* ctr, hipStream_t s) {
    hipLaunchKernelGGL(counters_reset_kernel, dim3(1), dim3(1), 0, s, ctr);
    return hipGetLastError();
}

// Thread per 32 tags (8 Philox blocks); a wave appends its hits with one
// atomic.  Tags are below 2^32.
__global__ __launch_bounds__(kT) void presample_kernel(uint64_t seed, uint64_t n, uint32_t round,
                                                       uint32_t thresh, uint32_t* __restrict__ list,
                                                       uint32_t cap, uint32_t* __restrict__ count) {
    const uint64_t words = (n + 31) / 32;
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    const uint32_t lane = lane_id();
    // every lane of a wave runs the same number of steps (the ballot and the
    // scan below need the whole wave)
    const uint64_t w0 = (uint64_t)blockIdx.x * kT + (threadIdx.x - lane);
    for (uint64_t wb = w0; wb < words; wb += stride) {
        const uint64_t w = wb + lane;
        uint32_t m = 0;
        if (w < words) {
#pragma unroll
            for (uint32_t i = 0; i < 8; ++i) {
                const Philox4 r = sample_block(seed, w * 8 + i, round);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (r.v[q] < thresh && w * 32 + i * 4 + q < n) m |= 1u << (i * 4 + q);
            }
        }
        if (__ballot(m != 0)) {
            const uint32_t c = __popc(m);
            const uint32_t inc = wave_inclusive_scan<uint32_t>(c);
            uint32_t base = 0;
            if (lane == kWave - 1) base = atomicAdd(count, inc);
            base = (uint32_t)__shfl((int)base, kWave - 1);
            uint32_t o = base + inc - c;
            while (m) {
                const uint32_t b = __ffs(m) - 1;
                m &= m - 1;
                if (o < cap) list[o] = (uint32_t)(w * 32 + b);
                ++o;
            }
        }
    }
}

__global__ void presample_reset_kernel(uint32_t* counts, uint32_t n) {
    if (threadIdx.x < n) counts[threadIdx.x] = 0;
}

hipError_t launch_presample_reset(uint32_t* counts, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(presample_reset_kernel, dim3(1), dim3(64), 0, s, counts, n);
    return hipGetLastError();
}

hipError_t launch_presample(uint64_t seed, uint64_t n, uint32_t round, uint32_t thresh, uint32_t* list,
                            uint32_t cap, uint32_t* count, hipStream_t s) {
    const uint64_t words = (n + 31) / 32;
    if (words == 0) return hipSuccess;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((words + kT - 1) / kT, 65536);
    hipLaunchKernelGGL(presample_kernel, dim3(grid), dim3(kT), 0, s, seed, n, round, thresh, list, cap,
                       count);
    return hipGetLastError();
}

hipError_t launch_round_init(const RoundArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(round_init_kernel, dim3(grid_for(a.n_rows, kT)), dim3(kT), 0, s, a);
    if (a.picks)
        hipLaunchKernelGGL(pick_clear_all_kernel, dim3(grid_for(a.pick_words, kT, 4096)), dim3(kT), 0, s,
                           a.pick_bits, a.pick_words);
    return hipGetLastError();
}

// at most one interval per splitter (rows minus the two ends of every instance)
static uint32_t interval_bound(const RoundArgs& a) {
    return a.n_rows > 2 * a.n_inst ? a.n_rows - 2 * a.n_inst : 1u;
}

hipError_t launch_round(const RoundArgs& a, uint32_t j, hipStream_t s, Profiler* prof) {
    const hipError_t e = launch_round_head(a, j, s);
    if (e != hipSuccess) return e;
    return launch_round_tail(a, j, s, false, prof);
}

hipError_t launch_round_head(const RoundArgs& a, uint32_t j, hipStream_t s) {
    const uint32_t ivl_bound = interval_bound(a);
    const bool small = a.n_rows <= kScanSmallRows;
    if (small) hipLaunchKernelGGL(leaders_kernel<kScanSmall>, dim3(1), dim3(kScanSmall), 0, s, a, j);
    else hipLaunchKernelGGL(leaders_kernel<kScanLarge>, dim3(1), dim3(kScanLarge), 0, s, a, j);
    hipLaunchKernelGGL(slices_kernel, dim3(ivl_bound), dim3(kT), 0, s, a);
    if (small) hipLaunchKernelGGL(ivl_scan_kernel<kScanSmall>, dim3(1), dim3(kScanSmall), 0, s, a);
    else hipLaunchKernelGGL(ivl_scan_kernel<kScanLarge>, dim3(1), dim3(kScanLarge), 0, s, a);
    hipLaunchKernelGGL(compact_kernel, dim3(ivl_bound), dim3(kT), 0, s, a);
    if (a.budget) hipLaunchKernelGGL(budget_rate_kernel, dim3(grid_for(a.n_inst, kT, 64)), dim3(kT), 0, s, a, j);
    if (a.n_inst == 1) {
        if (a.key_bytes == 4) hipLaunchKernelGGL((sample_kernel<uint32_t, true>), dim3(a.sample_grid), dim3(kT), 0, s, a, j);
        else hipLaunchKernelGGL((sample_kernel<uint64_t, true>), dim3(a.sample_grid), dim3(kT), 0, s, a, j);
    } else {
        if (a.key_bytes == 4) hipLaunchKernelGGL((sample_kernel<uint32_t, false>), dim3(a.sample_grid), dim3(kT), 0, s, a, j);
        else hipLaunchKernelGGL((sample_kernel<uint64_t, false>), dim3(a.sample_grid), dim3(kT), 0, s, a, j);
    }
    if (a.picks && a.n_inst == 1) {
        if (a.key_bytes == 4) hipLaunchKernelGGL(pick_sample_kernel<uint32_t>, dim3(a.sample_grid), dim3(kT), 0, s, a, j);
        else hipLaunchKernelGGL(pick_sample_kernel<uint64_t>, dim3(a.sample_grid), dim3(kT), 0, s, a, j);
    }
    if (small) hipLaunchKernelGGL(probe_scan_kernel<kScanSmall>, dim3(1), dim3(kScanSmall), 0, s, a, j);
    else hipLaunchKernelGGL(probe_scan_kernel<kScanLarge>, dim3(1), dim3(kScanLarge), 0, s, a, j);
    hipLaunchKernelGGL(group_kernel, dim3(grid_for(a.cap, kT, 4096)), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_round_tail(const RoundArgs& a, uint32_t j, hipStream_t s, bool probes_sorted,
                             Profiler* prof) {
    (void)prof;
    if (!probes_sorted) {
        const uint64_t tiles_bound = (a.cap + kOrderLanes - 1) / kOrderLanes + interval_bound(a);
        hipLaunchKernelGGL(order_kernel, dim3((unsigned)std::min<uint64_t>(tiles_bound, kOrderGrid)),
                           dim3(kOrderThreads), 0, s, a);
    }
    if (j == 1 && a.dense_rank && a.n_chunks > 0) {
        if (a.key_bytes == 4) hipLaunchKernelGGL(rank_dense_kernel<uint32_t>, dim3(a.n_chunks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(rank_dense_kernel<uint64_t>, dim3(a.n_chunks), dim3(256), 0, s, a);
    } else if (j >= a.pair_rank_from) {
        // every probe searched inside its own interval slice
        if (a.key_bytes == 4) hipLaunchKernelGGL(rank_pairs_kernel<uint32_t>, dim3(a.pair_grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(rank_pairs_kernel<uint64_t>, dim3(a.pair_grid), dim3(256), 0, s, a);
    } else if (a.n_chunks > 0) {
        if (a.key_bytes == 4) hipLaunchKernelGGL(rank_kernel<uint32_t>, dim3(a.n_chunks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL(rank_kernel<uint64_t>, dim3(a.n_chunks), dim3(256), 0, s, a);
    }
    const uint64_t rtiles = (a.cap + 255) / 256 * ((a.p_max + kReduceRows - 1) / kReduceRows);
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)std::min<uint64_t>(rtiles, kReduceGrid)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(settle_kernel<256>, dim3(a.n_rows), dim3(256), 0, s, a);
    const uint64_t copy_tiles = (uint64_t)((2 * a.n_rows + kCopySlots - 1) / kCopySlots) *
                                ((a.p_max + kCopySegs - 1) / kCopySegs);
    hipLaunchKernelGGL(settle_copy_kernel, dim3((unsigned)std::min<uint64_t>(copy_tiles, 16384)), dim3(256), 0, s, a);
    if (a.picks) hipLaunchKernelGGL(pick_clear_kernel, dim3(grid_for(a.cap, kT, 4096)), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_probe_offsets(const RoundArgs& a, uint64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(probe_offsets_kernel, dim3(grid_for(interval_bound(a) + 1, kT)), dim3(kT), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_probe_finish(const RoundArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(probe_finish_kernel, dim3(grid_for(a.cap, kT, 4096)), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const RoundArgs& a, uint64_t* chi_all, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(grid_for(a.n_rows, kT)), dim3(kT), 0, s, a, chi_all);
    return hipGetLastError();
}

hipError_t launch_segment_sources(const RoundArgs& a, const uint32_t* list, uint32_t count,
                                  uint64_t* key_src, uint64_t* val_src, int key_bytes,
                                  hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(segment_sources_kernel, dim3(grid_for(count, kT)), dim3(kT), 0, s, a, list,
                       count, key_src, val_src, key_bytes);
    return hipGetLastError();
}

hipError_t launch_set_run(const InstRun& r, InstRun* dst, hipStream_t s) {
    hipLaunchKernelGGL(set_run_kernel, dim3(1), dim3(1), 0, s, r, dst);
    return hipGetLastError();
}

}  // namespace hss
