// Splitter rounds of HSS (section 4.2.2, steps 1-5), all on the device.
//
// Round j, given the splitter state after round j-1:
//   intervals -- the distinct open intervals (L_i, U_i) of unsettled splitters
//                (identical intervals are taken once: they are either disjoint
//                or identical, section 4.2.2)
//   slices    -- per (interval, segment) the slice of the locally sorted
//                segment strictly inside the interval, as a run of 4-tag
//                Philox blocks in one flattened block space; the non-empty
//                slices are listed in (interval, segment) order
//   sample    -- every tag of the domain draws its Philox word and becomes a
//                probe when the word is below the round threshold
//                (section 4.2.1: independent Bernoulli with rate p s_j / N)
//   probe sort-- probes ordered by (key, tag), the strict order of section 6.1
//   rank      -- per probe, the number of keys of every segment that precede
//                it (the local histograms), summed over segments in the same
//                workgroup (the reduction of section 5.2)
//   settle    -- per unsettled splitter, a probe in its target range settles
//                it (closest to N i/p, lower rank on a tie); otherwise L and U
//                move to the closest probe ranks below and above N i/p
//   locate    -- per-segment counts of every new bound / splitter probe, which
//                become the next round's slice ends and the piece boundaries

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kT = 256;           // threads of most round kernels
constexpr int kSampleGrid = 4096; // workgroups of the grid-stride sampler
constexpr uint64_t kCountSortMax = 32768;   // probe sort by pairwise counting up to here
constexpr int kCountTile = 256;

__global__ void round_init_kernel(uint32_t p, uint32_t* settled, uint64_t* chi, uint64_t* lrank,
                                  uint64_t* urank, RoundCounters* ctr) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= p; i += gridDim.x * blockDim.x) {
        settled[i] = 0;
        chi[i] = 0;
        lrank[i] = kNone;
        urank[i] = kNone;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctr->m = 0;
        ctr->domain = 0;
        ctr->blocks = 0;
        ctr->n_ivl = 0;
        ctr->n_slices = 0;
        ctr->n_unsettled = 0;
        ctr->n_req = 0;
        ctr->err = 0;
    }
}

__global__ void counters_reset_kernel(RoundCounters* ctr) {
    *ctr = RoundCounters{};
}

// One workgroup: leaders of runs of identical unsettled intervals, in
// splitter order, compacted into ivl_row.
__global__ __launch_bounds__(1024) void leaders_kernel(RoundArgs a) {
    __shared__ uint32_t scratch[1024 / kWave];
    uint32_t base = 0, unsettled = 0;
    for (uint32_t c = 1; c < a.p; c += 1024) {
        const uint32_t i = c + threadIdx.x;
        const bool u = i < a.p && a.settled[i] == 0;
        bool lead = u;
        if (u && i > 1 && a.settled[i - 1] == 0 && a.lrank[i - 1] == a.lrank[i] &&
            a.urank[i - 1] == a.urank[i])
            lead = false;
        uint32_t tot;
        const uint32_t pre = block_exclusive_scan<uint32_t, 1024>(lead ? 1u : 0u, scratch, &tot);
        if (lead) a.ivl_row[base + pre] = i;
        base += tot;
        uint32_t ut;
        block_exclusive_scan<uint32_t, 1024>(u ? 1u : 0u, scratch, &ut);
        unsettled += ut;
    }
    if (threadIdx.x == 0) {
        a.ctr->n_ivl = base;
        a.ctr->n_unsettled = unsettled;
        a.ctr->m = 0;
        a.ctr->n_req = 0;
    }
}

__device__ __forceinline__ void slice_bounds(const RoundArgs& a, uint32_t row, uint32_t s,
                                             bool lnone, bool unone, uint64_t* ga, uint64_t* gb) {
    const uint64_t sb = a.seg_off[s];
    const uint64_t slen = a.seg_off[s + 1] - sb;
    const uint64_t lo = lnone ? 0 : a.lpos[(uint64_t)row * a.p + s];
    const uint64_t hi = unone ? slen : a.upos[(uint64_t)row * a.p + s];
    *ga = sb + lo;
    *gb = sb + (hi > lo ? hi : lo);
}

__device__ __forceinline__ uint64_t blocks_of(uint64_t ga, uint64_t gb) {
    return gb > ga ? ((gb - 1) >> 2) - (ga >> 2) + 1 : 0;
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

// Workgroup per interval k: Philox blocks, non-empty slices and tags of its
// p slices.
__global__ __launch_bounds__(kT) void slices_kernel(RoundArgs a) {
    __shared__ uint64_t scratch[kT / kWave];
    const uint32_t k = blockIdx.x;
    if (k >= a.ctr->n_ivl) return;
    const uint32_t row = a.ivl_row[k];
    const bool lnone = a.lrank[row] == kNone;
    const bool unone = a.urank[row] == kNone;
    uint64_t nb_sum = 0, nz_sum = 0, dom = 0;
    for (uint32_t s0 = 0; s0 < a.p; s0 += kT) {
        const uint32_t s = s0 + threadIdx.x;
        uint64_t nb = 0, len = 0;
        if (s < a.p) {
            uint64_t ga, gb;
            slice_bounds(a, row, s, lnone, unone, &ga, &gb);
            nb = blocks_of(ga, gb);
            len = gb - ga;
        }
        nb_sum += nb;
        nz_sum += nb ? 1 : 0;
        dom += len;
    }
    nb_sum = block_sum<uint64_t, kT>(nb_sum, scratch);
    nz_sum = block_sum<uint64_t, kT>(nz_sum, scratch);
    dom = block_sum<uint64_t, kT>(dom, scratch);
    if (threadIdx.x == 0) {
        a.ivl_tot[k] = nb_sum;
        a.ivl_nz[k] = (uint32_t)nz_sum;
        a.ivl_dom[k] = dom;
    }
}

// One workgroup: exclusive scans of the interval block and slice totals.
__global__ __launch_bounds__(1024) void ivl_scan_kernel(RoundArgs a) {
    __shared__ uint64_t scratch[1024 / kWave];
    const uint32_t n = a.ctr->n_ivl;
    uint64_t run = 0, run_nz = 0, dom = 0;
    for (uint32_t c = 0; c < n; c += 1024) {
        const uint32_t k = c + threadIdx.x;
        const uint64_t v = k < n ? a.ivl_tot[k] : 0;
        const uint64_t z = k < n ? a.ivl_nz[k] : 0;
        const uint64_t d = k < n ? a.ivl_dom[k] : 0;
        uint64_t tot, tot_nz;
        const uint64_t pre = block_exclusive_scan<uint64_t, 1024>(v, scratch, &tot);
        const uint64_t pre_nz = block_exclusive_scan<uint64_t, 1024>(z, scratch, &tot_nz);
        if (k < n) {
            a.ivl_tot[k] = run + pre;
            a.ivl_nz[k] = (uint32_t)(run_nz + pre_nz);
        }
        run += tot;
        run_nz += tot_nz;
        dom += block_sum<uint64_t, 1024>(d, scratch);
    }
    if (threadIdx.x == 0) {
        a.ivl_tot[n] = run;
        a.ivl_nz[n] = (uint32_t)run_nz;
        a.ctr->blocks = run;
        a.ctr->n_slices = (uint32_t)run_nz;
        a.ctr->domain = dom;
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
    const bool lnone = a.lrank[row] == kNone;
    const bool unone = a.urank[row] == kNone;
    uint64_t run = a.ivl_tot[k], run_nz = a.ivl_nz[k];
    for (uint32_t s0 = 0; s0 < a.p; s0 += kT) {
        const uint32_t s = s0 + threadIdx.x;
        uint64_t nb = 0, ga = 0, gb = 0;
        if (s < a.p) {
            slice_bounds(a, row, s, lnone, unone, &ga, &gb);
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

// Wave-per-range sampler.  Wave w of W takes the blocks [w T / W, (w+1) T / W)
// of the flattened block space (T blocks), one block per lane per step.  The
// slice list is walked with a window of 64 consecutive entries, one per lane:
// slices are non-empty, so the 64 blocks of a step lie in the 64 slices that
// start with the slice of the step's first block, and the next step's first
// block lies at most one slice past the window.
template <typename K>
__global__ __launch_bounds__(kT) void sample_kernel(RoundArgs a, uint64_t seed, uint32_t round,
                                                    uint32_t thresh, int take_all) {
    constexpr uint32_t kNoBlock = 0xFFFFFFFFu;   // start of the entries past the list
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
            // tags are below 2^32 (N < 2^32), so block and tag fit 32 bits
            const uint32_t blk32 = (ga >> 2) + (b - s_first);
            blk = blk32;
            const Philox4 r = sample_block(seed, blk, round);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (take_all || r.v[q] < thresh) hits |= 1u << q;
            // the first and last block of a slice may hold tags outside it
            const uint32_t g0 = blk32 * 4;
            if (g0 < ga || (uint64_t)g0 + 4 > gb) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (g0 + q < ga || g0 + q >= gb) hits &= ~(1u << q);
            }
        }
        if (__ballot(hits != 0)) {
            const uint32_t c = __popc(hits);
            const uint32_t inc = wave_inclusive_scan<uint32_t>(c);
            unsigned long long base = 0;
            if (lane == kWave - 1) base = atomicAdd(&a.ctr->m, (unsigned long long)inc);
            base = shfl_u64(base, kWave - 1);
            uint64_t o = base + inc - c;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (hits & (1u << q)) {
                    if (o < a.cap) {
                        const uint64_t g = blk * 4 + q;
                        a.pr_key[o] = (uint64_t)B[g];
                        a.pr_tag[o] = g;
                        a.pr_ivl[o] = k;
                        a.pr_pos[o] = 0;   // the probe sort counts into it
                    }
                    ++o;
                }
            }
        }
        e = en;
        nxt = nxtn;
        jq = jn;
    }
}

// Sorted position of every probe: the number of probes before it in the
// order (key, tag), counted against one tile of kCountTile probes per
// workgroup row.
__global__ __launch_bounds__(kT) void probe_count_kernel(const uint64_t* __restrict__ key,
                                                         const uint64_t* __restrict__ tag,
                                                         uint64_t m, uint32_t* __restrict__ pos) {
    __shared__ uint64_t sk[kCountTile];
    __shared__ uint64_t st[kCountTile];
    const uint64_t j0 = (uint64_t)blockIdx.y * kCountTile;
    const uint32_t nj = (uint32_t)min((uint64_t)kCountTile, m - j0);
    for (uint32_t j = threadIdx.x; j < nj; j += kT) {
        sk[j] = key[j0 + j];
        st[j] = tag[j0 + j];
    }
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    const uint64_t k = key[i], t = tag[i];
    uint32_t c = 0;
    for (uint32_t j = 0; j < nj; ++j) {
        const uint64_t kj = sk[j];
        c += (kj < k || (kj == k && st[j] < t)) ? 1u : 0u;
    }
    if (c) atomicAdd(&pos[i], c);
}

__device__ __forceinline__ uint32_t segment_of(const uint64_t* seg_off, uint32_t p, uint64_t g);

__global__ void probe_permute_kernel(RoundArgs a, uint64_t m, const uint64_t* order) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t src, dst;
        if (order) { src = order[i]; dst = i; }      // order[i] = emitted index of sorted i
        else { src = i; dst = a.pr_pos[i]; }          // pr_pos[i] = sorted index of emitted i
        const uint64_t g = a.pr_tag[src];
        a.ps_key[dst] = a.pr_key[src];
        a.ps_tag[dst] = g;
        a.ps_ivl[dst] = a.pr_ivl[src];
        a.ps_seg[dst] = segment_of(a.seg_off, a.p, g);
        a.pr_rank[dst] = 0;   // the rank reduction adds into it
    }
}

__global__ void iota_kernel(uint64_t* v, uint64_t m) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x)
        v[i] = i;
}

__global__ void gather_kernel(const uint64_t* __restrict__ src, const uint64_t* __restrict__ idx,
                              uint64_t* __restrict__ dst, uint64_t m) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

__global__ void one_segment_kernel(uint64_t* seg, uint64_t m) {
    seg[0] = 0;
    seg[1] = m;
}

__device__ __forceinline__ uint32_t segment_of(const uint64_t* seg_off, uint32_t p, uint64_t g) {
    return last_le(seg_off, p + 1, g);
}

// Workgroup per sorted probe: c_s for every segment s inside the slice of the
// probe's own interval, summed -> R(e).  One segment per thread (kThreads =
// 1024 when p is large, so that many dependent searches are in flight per CU).
// With a count matrix, c_s(e) is also stored at cmat[e * p + s] for locate.
template <typename K, int kThreads>
__global__ __launch_bounds__(kThreads) void rank_kernel(RoundArgs a, uint32_t* __restrict__ cmat) {
    __shared__ uint64_t scratch[kThreads / kWave];
    __shared__ uint32_t sh_t;
    const uint64_t e = blockIdx.x;
    const K key = (K)a.ps_key[e];
    const uint64_t g = a.ps_tag[e];
    const uint32_t row = a.ivl_row[a.ps_ivl[e]];
    if (threadIdx.x == 0) sh_t = segment_of(a.seg_off, a.p, g);
    __syncthreads();
    const uint32_t t = sh_t;
    const bool lnone = a.lrank[row] == kNone;
    const bool unone = a.urank[row] == kNone;
    const K* B = (const K*)a.B;
    uint64_t sum = 0;
    for (uint32_t s = threadIdx.x; s < a.p; s += kThreads) {
        const uint64_t sb = a.seg_off[s];
        const uint64_t slen = a.seg_off[s + 1] - sb;
        const uint64_t lo = lnone ? 0 : a.lpos[(uint64_t)row * a.p + s];
        const uint64_t hi = unone ? slen : a.upos[(uint64_t)row * a.p + s];
        uint64_t c;
        if (s == t) {
            c = g - sb;
            if (c < lo || c >= hi) atomicOr(&a.ctr->err, kErrProbeOutside);
        } else {
            // equal keys of earlier segments precede the probe, of later ones follow
            c = count_before<K>(B + sb, lo, hi, key, s < t);
        }
        sum += c;
        if (cmat) cmat[(uint64_t)s * gridDim.x + e] = (uint32_t)c;
    }
    sum = block_sum<uint64_t, kThreads>(sum, scratch);
    if (threadIdx.x == 0) a.pr_rank[e] = sum;
}

constexpr uint32_t kRankChunk = 1u << 15;                  // keys of a segment per workgroup
constexpr uint32_t kRankFences = kRankChunk / kFenceStride;  // their fences, held in LDS

// (key_e, g_e) after (kx, gx) in the order (key, tag)?
template <typename K>
__device__ __forceinline__ bool after(K ke, uint64_t ge, K kx, uint64_t gx) {
    return ke > kx || (ke == kx && ge > gx);
}

// Workgroup per (segment s, chunk c): the probes e whose count c_s(e) falls
// in the chunk are the sorted run [e0, e1); each finds its place among the
// chunk's fences in LDS, then inside one kFenceStride-key block of B.
// Result: cmat[s * m + e] = c_s(e).
template <typename K>
__global__ __launch_bounds__(256) void rank_seg_kernel(RoundArgs a, uint64_t m,
                                                       uint32_t chunks_per_seg, Fences fn,
                                                       uint32_t* __restrict__ cmat) {
    __shared__ uint64_t F[kRankFences];
    __shared__ uint64_t sh_e[2];
    __shared__ uint32_t sh_cnt[2];
    const uint32_t s = blockIdx.x / chunks_per_seg;
    const uint32_t c = blockIdx.x % chunks_per_seg;
    const uint64_t sb = a.seg_off[s];
    const uint64_t ns = a.seg_off[s + 1] - sb;
    const uint32_t nchunks = ns == 0 ? 1u : (uint32_t)((ns + kRankChunk - 1) / kRankChunk);
    if (c >= nchunks) return;
    const bool last = c + 1 == nchunks;
    const uint64_t lo_pos = (uint64_t)c * kRankChunk;
    const uint64_t chunk_end = min(lo_pos + kRankChunk, ns);   // last element + 1 in the chunk
    const K* B = (const K*)a.B + sb;
    // [e0, e1): the probes with c_s(e) in the chunk.  The first probe with
    // c_s(e) >= x (x >= 1) is the first probe after the element at position
    // x - 1 of the segment.  Two parallel steps: 256 evenly spaced probes
    // bracket the answer, then every probe of the bracket is tested.
    const bool need0 = lo_pos != 0, need1 = !last;
    // no probe after the boundary element: m; no boundary (first chunk): 0
    if (threadIdx.x < 2) sh_e[threadIdx.x] = (threadIdx.x == 0 && !need0) ? 0 : m;
    if (threadIdx.x == 0) sh_cnt[0] = sh_cnt[1] = 0;
    __syncthreads();
    const uint64_t step = (m + 255) / 256;
    K bx[2];
    uint64_t bg[2];
    bx[0] = need0 ? B[lo_pos - 1] : (K)0;
    bg[0] = sb + lo_pos - 1;
    bx[1] = need1 ? B[chunk_end - 1] : (K)0;
    bg[1] = sb + chunk_end - 1;
    {
        // probes j*step before or at each boundary element (j = 0..255)
        const uint64_t j = (uint64_t)threadIdx.x * step;
        if (j < m) {
            const K kj = (K)a.ps_key[j];
            const uint64_t gj = a.ps_tag[j];
            if (need0 && !after<K>(kj, gj, bx[0], bg[0])) atomicAdd(&sh_cnt[0], 1u);
            if (need1 && !after<K>(kj, gj, bx[1], bg[1])) atomicAdd(&sh_cnt[1], 1u);
        }
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
        if (!(q == 0 ? need0 : need1)) continue;   // uniform
        // c samples are not after the boundary (the predicate is monotone over
        // the sorted probes), so the answer lies in [(c-1)*step + 1, c*step],
        // or is m when no probe of that range is after it
        const uint64_t c = sh_cnt[q];
        const uint64_t lo = c == 0 ? 0 : (c - 1) * step + 1;
        const uint64_t hi = min(c * step + 1, m);   // exclusive
        for (uint64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
            if (after<K>((K)a.ps_key[e], a.ps_tag[e], bx[q], bg[q]) &&
                (e == 0 || !after<K>((K)a.ps_key[e - 1], a.ps_tag[e - 1], bx[q], bg[q])))
                sh_e[q] = e;   // exactly one e qualifies
        }
    }
    __syncthreads();
    const uint64_t e0 = sh_e[0], e1 = sh_e[1];
    if (e0 >= e1) return;   // no probe counts into this chunk (uniform over the workgroup)
    const uint32_t nf = (uint32_t)((chunk_end - lo_pos + kFenceStride - 1) / kFenceStride);
    const uint64_t* fsrc = fn.key + (uint64_t)s * fn.per_seg + lo_pos / kFenceStride;
    for (uint32_t i = threadIdx.x; i < nf; i += blockDim.x) F[i] = fsrc[i];
    __syncthreads();
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const K key = (K)a.ps_key[e];
        const uint64_t g = a.ps_tag[e];
        const uint32_t t = a.ps_seg[e];
        uint64_t cnt;
        if (t == s) {
            cnt = g - sb;
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
        cmat[(uint64_t)s * m + e] = (uint32_t)cnt;
    }
}

constexpr uint32_t kReduceRows = 16;   // segments summed per workgroup of the reduction

// The reduction of section 5.2: R(e) is the sum over segments of c_s(e), the
// column sums of the count matrix.  Tiles of 256 probes x kReduceRows
// segments; the partial sums are integers, so the order of the atomic
// additions does not change R(e).
__global__ __launch_bounds__(256) void rank_reduce_kernel(const uint32_t* __restrict__ cmat,
                                                          uint64_t m, uint32_t p,
                                                          uint64_t* __restrict__ pr_rank) {
    const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m) return;
    const uint32_t s0 = blockIdx.y * kReduceRows;
    const uint32_t s1 = min(s0 + kReduceRows, p);
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t s = s0; s < s1; ++s) sum += cmat[(uint64_t)s * m + e];
    atomicAdd((unsigned long long*)&pr_rank[e], (unsigned long long)sum);
}

__device__ __forceinline__ void emit_request(const RoundArgs& a, uint32_t e, uint32_t row,
                                             uint32_t kind) {
    const uint32_t r = atomicAdd(&a.ctr->n_req, 1u);
    a.req_probe[r] = e;
    a.req_row[r] = row;
    a.req_kind[r] = kind;
}

// Thread per splitter i = 1..p-1.
__global__ __launch_bounds__(kT) void settle_kernel(RoundArgs a, uint64_t m) {
    const uint64_t gid = (uint64_t)blockIdx.x * kT + threadIdx.x;
    for (uint64_t e = gid; e + 1 < m; e += (uint64_t)gridDim.x * kT)
        if (a.pr_rank[e] >= a.pr_rank[e + 1]) atomicOr(&a.ctr->err, kErrRankOrder);
    const uint64_t i = gid + 1;
    if (i >= a.p || a.settled[i]) return;
    const uint64_t target = a.ideal[i];
    // first probe with R >= N i / p
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a.pr_rank[mid] < target) lo = mid + 1; else hi = mid;
    }
    const bool has_above = lo < m;
    const bool has_below = lo > 0;
    const uint64_t r_above = has_above ? a.pr_rank[lo] : 0;
    const uint64_t r_below = has_below ? a.pr_rank[lo - 1] : 0;
    const uint64_t d_above = r_above - target;
    const uint64_t d_below = target - r_below;
    int64_t pick = -1;
    if (has_below && d_below <= a.tol) pick = (int64_t)lo - 1;
    if (has_above && d_above <= a.tol && (pick < 0 || d_above < d_below)) pick = (int64_t)lo;
    if (pick >= 0) {
        a.settled[i] = 1;
        a.chi[i] = a.pr_rank[pick];
        a.s_key[i] = a.ps_key[pick];
        a.s_tag[i] = a.ps_tag[pick];
        emit_request(a, (uint32_t)pick, (uint32_t)i, 2u);
        return;
    }
    if (has_below && (a.lrank[i] == kNone || r_below > a.lrank[i])) {
        a.lrank[i] = r_below;
        emit_request(a, (uint32_t)(lo - 1), (uint32_t)i, 0u);
    }
    if (has_above && r_above < a.urank[i]) {
        a.urank[i] = r_above;
        emit_request(a, (uint32_t)lo, (uint32_t)i, 1u);
    }
}

// Workgroup per request: per-segment counts of a new bound / splitter probe,
// copied from the rank step's count matrix or found by searching each segment.
template <typename K, int kThreads>
__global__ __launch_bounds__(kThreads) void locate_kernel(RoundArgs a,
                                                          const uint32_t* __restrict__ cmat,
                                                          uint64_t m) {
    __shared__ uint32_t sh_t;
    const uint32_t r = blockIdx.x;
    if (r >= a.ctr->n_req) return;
    const uint32_t e = a.req_probe[r];
    const uint64_t row = a.req_row[r];
    const uint32_t kind = a.req_kind[r];
    const K key = (K)a.ps_key[e];
    const uint64_t g = a.ps_tag[e];
    if (threadIdx.x == 0) sh_t = segment_of(a.seg_off, a.p, g);
    __syncthreads();
    const uint32_t t = sh_t;
    const K* B = (const K*)a.B;
    uint32_t* dst = kind == 0 ? a.lpos : (kind == 1 ? a.upos : a.prow);
    const uint32_t own = kind == 0 ? 1u : 0u;   // the L probe itself is excluded
    for (uint32_t s = threadIdx.x; s < a.p; s += kThreads) {
        uint64_t c;
        if (cmat) {
            c = cmat[(uint64_t)s * m + e];
        } else {
            const uint64_t sb = a.seg_off[s];
            c = s == t ? g - sb : count_before<K>(B + sb, 0, a.seg_off[s + 1] - sb, key, s < t);
        }
        dst[row * a.p + s] = (uint32_t)c + (s == t ? own : 0u);
    }
}

__global__ void finalize_kernel(RoundArgs a, uint64_t* offsets) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= a.p; i += gridDim.x * blockDim.x)
        offsets[i] = i == 0 ? 0 : (i == a.p ? a.n : a.chi[i]);
}

unsigned grid_for(uint64_t n, unsigned threads, unsigned cap = 65535u) {
    const uint64_t g = (n + threads - 1) / threads;
    return (unsigned)(g == 0 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_round_init(const RoundArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(round_init_kernel, dim3(grid_for(a.p + 1, kT)), dim3(kT), 0, s, a.p,
                       a.settled, a.chi, a.lrank, a.urank, a.ctr);
    return hipGetLastError();
}

hipError_t launch_counters_reset(RoundCounters* ctr, hipStream_t s) {
    hipLaunchKernelGGL(counters_reset_kernel, dim3(1), dim3(1), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_intervals(const RoundArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(leaders_kernel, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(slices_kernel, dim3(a.p > 1 ? a.p - 1 : 1), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(ivl_scan_kernel, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(compact_kernel, dim3(a.p > 1 ? a.p - 1 : 1), dim3(kT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sample(const RoundArgs& a, uint64_t seed, uint32_t round, uint32_t thresh,
                         int take_all, hipStream_t s) {
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(sample_kernel<uint32_t>, dim3(kSampleGrid), dim3(kT), 0, s, a, seed,
                           round, thresh, take_all);
    else
        hipLaunchKernelGGL(sample_kernel<uint64_t>, dim3(kSampleGrid), dim3(kT), 0, s, a, seed,
                           round, thresh, take_all);
    return hipGetLastError();
}

size_t probe_sort_scratch_bytes(uint64_t m) {
    if (m <= kCountSortMax) return 0;
    // seg(2) + idx + idx_tmp + key_a + key_b, 8 bytes each
    return 16 + 4 * m * 8 + 256;
}

hipError_t launch_probe_sort(const RoundArgs& a, uint64_t m, void* scratch, size_t scratch_bytes,
                             uint32_t* counts, hipStream_t s) {
    if (m == 0) return hipSuccess;
    if (m <= kCountSortMax) {
        dim3 grid((unsigned)((m + kT - 1) / kT), (unsigned)((m + kCountTile - 1) / kCountTile));
        hipLaunchKernelGGL(probe_count_kernel, grid, dim3(kT), 0, s, a.pr_key, a.pr_tag, m,
                           a.pr_pos);
        hipLaunchKernelGGL(probe_permute_kernel, dim3(grid_for(m, kT)), dim3(kT), 0, s, a, m,
                           (const uint64_t*)nullptr);
        return hipGetLastError();
    }
    if (scratch_bytes < probe_sort_scratch_bytes(m)) return hipErrorInvalidValue;
    // Two stable LSD sorts: by tag, then by key -> order (key, tag).
    uint64_t* seg = (uint64_t*)scratch;
    uint64_t* idx = seg + 2;
    uint64_t* idx_tmp = idx + m;
    uint64_t* ka = idx_tmp + m;
    uint64_t* kb = ka + m;
    hipLaunchKernelGGL(one_segment_kernel, dim3(1), dim3(1), 0, s, seg, m);
    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(m, kT)), dim3(kT), 0, s, ka, m);
    SegSort ss;
    ss.key_bytes = 8;
    ss.seg_off = seg;
    ss.num_segs = 1;
    ss.max_seg_len = m;
    ss.counts = counts;
    // by tag: keys = tags, payload = emitted index
    ss.keys_in = a.pr_tag;
    ss.vals_in = ka;
    ss.keys_out = kb;
    ss.vals_out = idx;
    ss.keys_tmp = a.ps_tag;          // free until the permute below
    ss.vals_tmp = idx_tmp;
    ss.begin_bit = 0;
    ss.end_bit = 64;
    hipError_t err = segmented_radix_sort(ss, s);
    if (err != hipSuccess) return err;
    // by key, stably: keys = key of each index in tag order
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(m, kT)), dim3(kT), 0, s, a.pr_key, idx, ka, m);
    ss.keys_in = ka;
    ss.vals_in = idx;
    ss.keys_out = kb;
    ss.vals_out = idx_tmp;
    ss.keys_tmp = a.ps_key;
    ss.vals_tmp = a.ps_tag;
    ss.end_bit = a.key_bytes * 8;
    err = segmented_radix_sort(ss, s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(probe_permute_kernel, dim3(grid_for(m, kT)), dim3(kT), 0, s, a, m,
                       (const uint64_t*)idx_tmp);
    return hipGetLastError();
}

hipError_t launch_rank(const RoundArgs& a, uint64_t m, uint32_t* cmat, const Fences& fences,
                       uint64_t max_seg, hipStream_t s) {
    if (m == 0) return hipSuccess;
    if (cmat && fences.key) {
        const uint32_t cps = max_seg == 0 ? 1u : (uint32_t)((max_seg + kRankChunk - 1) / kRankChunk);
        const dim3 grid((unsigned)((uint64_t)a.p * cps));
        if (a.key_bytes == 4) hipLaunchKernelGGL(rank_seg_kernel<uint32_t>, grid, dim3(256), 0, s, a, m, cps, fences, cmat);
        else hipLaunchKernelGGL(rank_seg_kernel<uint64_t>, grid, dim3(256), 0, s, a, m, cps, fences, cmat);
        const dim3 rgrid((unsigned)((m + 255) / 256), (a.p + kReduceRows - 1) / kReduceRows);
        hipLaunchKernelGGL(rank_reduce_kernel, rgrid, dim3(256), 0, s, (const uint32_t*)cmat, m, a.p, a.pr_rank);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)m);
    if (a.p > 256) {
        if (a.key_bytes == 4) hipLaunchKernelGGL((rank_kernel<uint32_t, 1024>), grid, dim3(1024), 0, s, a, cmat);
        else hipLaunchKernelGGL((rank_kernel<uint64_t, 1024>), grid, dim3(1024), 0, s, a, cmat);
    } else {
        if (a.key_bytes == 4) hipLaunchKernelGGL((rank_kernel<uint32_t, 256>), grid, dim3(256), 0, s, a, cmat);
        else hipLaunchKernelGGL((rank_kernel<uint64_t, 256>), grid, dim3(256), 0, s, a, cmat);
    }
    return hipGetLastError();
}

hipError_t launch_settle(const RoundArgs& a, uint64_t m, hipStream_t s) {
    hipLaunchKernelGGL(settle_kernel, dim3(grid_for(a.p, kT)), dim3(kT), 0, s, a, m);
    return hipGetLastError();
}

hipError_t launch_locate(const RoundArgs& a, const uint32_t* cmat, uint64_t m, hipStream_t s) {
    const dim3 grid(2u * (a.p > 1 ? a.p - 1 : 1));
    if (a.p > 256) {
        if (a.key_bytes == 4) hipLaunchKernelGGL((locate_kernel<uint32_t, 1024>), grid, dim3(1024), 0, s, a, cmat, m);
        else hipLaunchKernelGGL((locate_kernel<uint64_t, 1024>), grid, dim3(1024), 0, s, a, cmat, m);
    } else {
        if (a.key_bytes == 4) hipLaunchKernelGGL((locate_kernel<uint32_t, 256>), grid, dim3(256), 0, s, a, cmat, m);
        else hipLaunchKernelGGL((locate_kernel<uint64_t, 256>), grid, dim3(256), 0, s, a, cmat, m);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const RoundArgs& a, uint64_t* d_offsets, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(grid_for(a.p + 1, kT)), dim3(kT), 0, s, a, d_offsets);
    return hipGetLastError();
}

}  // namespace hss
