// CPU oracle for Histogram Sort with Sampling (Harsh, Kale, Solomonik, SPAA'19).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
// statement of what the GPU path must compute.  Only the test-suite, the smoke
// check and the CPU-baseline leg of the benchmark load it.  It shares no code,
// header, table or constant with the HIP library, and the HIP library never
// calls it.
//
// Everything here follows the paper's notation:
//   N keys in p segments ("processors"), tolerance eps, splitters i = 1..p-1,
//   target range T_i around the ideal rank N*i/p (section 2),
//   rounds j = 1, 2, ... with sampling ratio s_j (section 4.2),
//   splitter interval [L_j(i), U_j(i)] and their union gamma_j (Table 1),
//   keys made distinct by the implicit tag (key, segment, index) (section 6.1).
//
// Readings of points the paper leaves open are marked READING and collected
// in the design notes of the repository.
//
// Parity status of each exported function is stated beside it.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <thread>
#include <utility>
#include <vector>

namespace {

typedef unsigned __int128 u128;

// ---------------------------------------------------------------------------
// Work over the p processors (segments) may be split among host threads: the
// paper's processors do it concurrently, every segment's share is computed
// on its own, and whatever is added up across segments is an integer sum,
// whose value does not depend on the order.  Thread t takes the contiguous
// range of items [t n / T, (t+1) n / T); f(t, lo, hi) runs once per thread.
// ---------------------------------------------------------------------------
template <typename F>
void split_over(uint64_t n, int threads, F f) {
    int T = threads < 1 ? 1 : threads;
    if ((uint64_t)T > n) T = n == 0 ? 1 : (int)n;
    if (T == 1) { f(0, (uint64_t)0, n); return; }
    std::vector<std::thread> pool;
    for (int t = 0; t < T; ++t) {
        uint64_t lo = (uint64_t)(((u128)t * n) / (u128)T);
        uint64_t hi = (uint64_t)(((u128)(t + 1) * n) / (u128)T);
        pool.emplace_back([=, &f]() { f(t, lo, hi); });
    }
    for (auto& th : pool) th.join();
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// Philox4x32-10, written from Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3" (SC'11): a 4-word counter, a 2-word key,
// ten rounds of two 32x32->64 multiplies, with the key advanced by the two
// Weyl constants between rounds.
// Pinned against rocRAND's independent implementation in the tests.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t prod0 = (uint64_t)M0 * x0;
        uint64_t prod1 = (uint64_t)M1 * x2;
        uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod1;
        uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

// The random word that decides whether the element with tag g is a probe in
// round j (READING: the paper does not fix a generator; the counter is
// (g div 4, j, 0) and the word is g mod 4 of the block).
uint32_t philox_word(uint64_t seed, uint64_t g, uint32_t j) {
    uint64_t blk = g >> 2;
    uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), j, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    philox4x32_10(ctr, key, out);
    return out[g & 3];
}

// ---------------------------------------------------------------------------
// Round constants (section 2 target range; section 4.2 rate schedule
// s_j = (2 ln p / eps)^(j/k); section 4.2 choice k = log(log p / eps)).
// ---------------------------------------------------------------------------
struct Constants {
    uint64_t tol;        // half-width of the target range, floor(N eps / (2p))
    uint32_t k;          // number of rounds of the schedule
    double a;            // 2 ln p / eps, the final sampling ratio s_k
};

Constants make_constants(uint64_t n, uint32_t p, double eps, uint32_t k_override) {
    Constants c;
    // READING: the target range is [Ni/p - N eps/(2p), Ni/p + N eps/(2p)]
    // (section 2), rounded down to an integer half-width.
    c.tol = (uint64_t)std::floor(((double)n * eps) / (2.0 * (double)p));
    // s_k = 2 ln p / eps is the ratio of the final round (lemma on the k-th
    // round and the one-round lemma of section 4.1).
    c.a = 2.0 * std::log((double)p) / eps;
    // READING: k = log(log p / eps) with natural logarithms, made the integer
    // ceil(ln a) so that s_k = a exactly; at least one round.
    double lk = std::ceil(std::log(c.a));
    c.k = lk < 1.0 ? 1u : (uint32_t)lk;
    if (k_override) c.k = k_override;
    return c;
}

// Sampling rate of round j: each key of gamma_{j-1} is a probe with
// probability p s_j / N (section 4.2.1).  READING: rounds after the k-th keep
// the same geometric schedule, and the probability is clamped at 1.
// Returns true when every key of the domain is taken; else *thresh is the
// 32-bit acceptance threshold floor(q * 2^32).
bool sampling_threshold(uint64_t n, uint32_t p, const Constants& c, uint32_t j,
                        uint32_t* thresh) {
    double s_j = std::pow(c.a, (double)j / (double)c.k);
    double q = ((double)p * s_j) / (double)n;
    if (q >= 1.0) { *thresh = 0xFFFFFFFFu; return true; }
    *thresh = (uint32_t)std::floor(q * 4294967296.0);
    return false;
}

// Fixed probe budget (the implementation of section 6, and the theorem with
// O(p) samples per round): c p probes per round in expectation.  READING:
// each key of the domain gamma_{j-1} is a probe with probability
// c p / |gamma_{j-1}|, clamped at 1, in place of the schedule p s_j / N; the
// same acceptance threshold floor(q 2^32) as above.
bool budget_threshold(uint64_t domain, uint32_t p, uint32_t c, uint32_t* thresh) {
    double q = ((double)c * (double)p) / (double)domain;
    if (q >= 1.0) { *thresh = 0xFFFFFFFFu; return true; }
    *thresh = (uint32_t)std::floor(q * 4294967296.0);
    return false;
}

// The implementation of section 6 with s = c probes per processor: when the
// splitter intervals cover the fraction delta = |gamma| / N of the input,
// every processor picks c / delta keys from its whole (sorted) input and
// discards those outside the intervals, so c p probes are kept in
// expectation.  READING: the picks are uniform positions of the processor's
// segment, drawn with replacement (a position picked twice is one probe);
// their number is ceil(c N / |gamma|), computed in double; once it reaches
// the largest segment every key of the intervals is taken instead (the
// analogue of a rate of 1).  Returns true in that case, else *picks.
bool pick_count(uint64_t n, uint64_t max_seg, uint64_t domain, uint32_t c, uint32_t* picks) {
    double d = std::ceil(((double)c * (double)n) / (double)domain);
    if (d >= (double)max_seg) { *picks = 0xFFFFFFFFu; return true; }
    *picks = (uint32_t)d;
    return false;
}

// Pick l of segment s in round j: a uniform position of the segment's n_s
// keys from a 32-bit Philox word, floor(word n_s / 2^32).  READING: the
// counter is (l, s, j, 1) (the last word 1 keeps these draws apart from
// the per-key draws), the word is the block's first.
uint64_t pick_position(uint64_t seed, uint32_t l, uint32_t s, uint32_t j, uint64_t n_s) {
    uint32_t ctr[4] = {l, s, j, 1u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    philox4x32_10(ctr, key, out);
    return (uint64_t)(((u128)out[0] * (u128)n_s) >> 32);
}

// Ideal rank N i / p of splitter i, exact (section 2).
uint64_t ideal_rank(uint64_t n, uint32_t p, uint64_t i) {
    return (uint64_t)(((u128)i * (u128)n) / (u128)p);
}

// ---------------------------------------------------------------------------
// One element of the locally sorted buffer: its key, its payload and its tag
// g (position in the buffer).  The strict order of section 6.1 is (key, g).
// ---------------------------------------------------------------------------
struct Problem {
    uint64_t n;
    uint32_t p;
    std::vector<uint64_t> seg_start;   // p+1 boundaries floor(s N / p)
    std::vector<uint64_t> key;         // B: keys sorted stably inside each segment
    std::vector<uint64_t> val;         // payload permuted with the keys

    uint32_t segment_of(uint64_t g) const {
        // largest s with seg_start[s] <= g
        auto it = std::upper_bound(seg_start.begin(), seg_start.end(), g);
        return (uint32_t)((it - seg_start.begin()) - 1);
    }
    uint64_t seg_len(uint32_t s) const { return seg_start[s + 1] - seg_start[s]; }

    // c_s(e): number of elements of segment s that precede the element with
    // tag g in the order (key, segment, index) of section 6.1.
    uint64_t count_below(uint32_t s, uint64_t g) const {
        uint32_t t = segment_of(g);
        if (s == t) return g - seg_start[t];
        const uint64_t* b = key.data() + seg_start[s];
        const uint64_t* e = key.data() + seg_start[s + 1];
        uint64_t kv = key[g];
        if (s < t) return (uint64_t)(std::upper_bound(b, e, kv) - b);   // equal keys of earlier segments precede
        return (uint64_t)(std::lower_bound(b, e, kv) - b);              // equal keys of later segments follow
    }
    uint64_t rank(uint64_t g) const {
        uint64_t r = 0;
        for (uint32_t s = 0; s < p; ++s) r += count_below(s, g);
        return r;
    }
};

const uint64_t NONE = ~(uint64_t)0;

struct Splitter {
    bool settled = false;
    uint64_t chi = 0;        // settled rank chi(i)
    uint64_t S = NONE;       // tag of the settled splitter key S(i)
    uint64_t L = NONE;       // tag of the bounding probe below (NONE = -infinity)
    uint64_t Lrank = 0;      // its rank (meaningful when L != NONE)
    uint64_t U = NONE;       // tag of the bounding probe above (NONE = +infinity)
    uint64_t Urank = 0;
};

struct RoundTrace {
    uint64_t domain = 0;                 // |gamma_{j-1}| as sampled (distinct elements)
    uint32_t thresh = 0;                 // acceptance threshold (0xFFFFFFFF with all=1)
    uint32_t all = 0;
    std::vector<uint64_t> probe_key;     // probes sorted by (key, g)
    std::vector<uint64_t> probe_tag;
    std::vector<uint64_t> probe_rank;    // R(e)
    std::vector<uint32_t> counts;        // c_s(e), probe-major, only with trace level >= 2
    std::vector<uint64_t> lo_rank;       // after the round: L rank per splitter (NONE = -inf)
    std::vector<uint64_t> hi_rank;       // after the round: U rank per splitter (NONE = +inf)
    std::vector<uint8_t> settled;        // after the round
    std::vector<uint64_t> chi;           // after the round (0 where unsettled)
};

struct Run {
    int status = 0;
    Constants c{};
    std::vector<RoundTrace> rounds;
    std::vector<uint64_t> chi;           // q+1 (q buckets, q = p but in a stage)
    std::vector<uint64_t> S_key, S_tag;  // q+1 (entries 0 and q unused)
    std::vector<uint64_t> pieces;        // (q+1) x p, row b holds c_s(S(b))
    double t_local = 0, t_rounds = 0, t_exchange = 0, t_final = 0;
};

}  // namespace

// ===========================================================================
// Exported interface (ctypes).  Status codes follow the library's header:
// 0 ok, -1 invalid argument, -5 round cap reached.
// ===========================================================================
extern "C" {

struct oracle_run;   // opaque: a Run

// Philox4x32-10 block function.  Pinned: rocRAND's philox engine.
void oracle_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
}

// Constants of a plan.  thresh_out[j-1], all_out[j-1] for j = 1..max_j.
// Pinned: closed forms of section 4.2 and the worked numbers of section 7.2.
void oracle_constants(uint64_t n, uint32_t p, double eps, uint32_t k_override,
                      uint64_t* tol, uint32_t* k, double* a, uint32_t max_j,
                      uint32_t* thresh_out, uint32_t* all_out) {
    Constants c = make_constants(n, p, eps, k_override);
    *tol = c.tol; *k = c.k; *a = c.a;
    for (uint32_t j = 1; j <= max_j; ++j) {
        uint32_t t;
        bool all = sampling_threshold(n, p, c, j, &t);
        thresh_out[j - 1] = t;
        all_out[j - 1] = all ? 1u : 0u;
    }
}

// The per-element probe decision word (exported so that the sampling
// statistics can be tested directly).
uint32_t oracle_philox_word(uint64_t seed, uint64_t g, uint32_t j) {
    return philox_word(seed, g, j);
}

}  // extern "C"

namespace {

// Parameters valid for the method (section 2: every segment gets N/p keys,
// so 1 <= p <= N; 0 < eps < 1 keeps the target ranges apart).
bool valid_params(uint64_t n, uint32_t p, double eps, int key_bits) {
    if (n == 0 || p == 0 || (uint64_t)p > n) return false;
    if (!(eps > 0.0 && eps < 1.0)) return false;
    if (key_bits != 32 && key_bits != 64) return false;
    return true;
}

void load_and_local_sort(Problem& P, uint64_t n, uint32_t p, int key_bits,
                         const void* keys_in, const uint64_t* vals_in, int threads) {
    P.n = n; P.p = p;
    P.seg_start.resize(p + 1);
    for (uint64_t s = 0; s <= p; ++s) P.seg_start[s] = (uint64_t)(((u128)s * n) / p);
    P.key.resize(n);
    P.val.resize(n);
    // Local sort of each segment (section 6: phase 1), stable so that the tag
    // order inside a segment is the input order among equal keys.  Every
    // processor loads and sorts its own segment.
    split_over(p, threads, [&](int, uint64_t s0, uint64_t s1) {
        for (uint64_t s = s0; s < s1; ++s) {
            uint64_t b = P.seg_start[s], e = P.seg_start[s + 1];
            for (uint64_t i = b; i < e; ++i) {
                P.key[i] = key_bits == 32 ? (uint64_t)((const uint32_t*)keys_in)[i]
                                          : ((const uint64_t*)keys_in)[i];
                P.val[i] = vals_in ? vals_in[i] : 0;
            }
            std::vector<uint64_t> idx(e - b);
            std::iota(idx.begin(), idx.end(), b);
            std::stable_sort(idx.begin(), idx.end(),
                             [&](uint64_t x, uint64_t y) { return P.key[x] < P.key[y]; });
            std::vector<uint64_t> k2(e - b), v2(e - b);
            for (uint64_t t = 0; t < e - b; ++t) { k2[t] = P.key[idx[t]]; v2[t] = P.val[idx[t]]; }
            std::copy(k2.begin(), k2.end(), P.key.begin() + b);
            std::copy(v2.begin(), v2.end(), P.val.begin() + b);
        }
    });
}

// Strict order of section 6.1 on tags of the locally sorted buffer.
bool before(const Problem& P, uint64_t g1, uint64_t g2) {
    if (P.key[g1] != P.key[g2]) return P.key[g1] < P.key[g2];
    return g1 < g2;
}

// Splitter determination by k-round HSS (section 4.2.2, steps 1-5), with the
// early stop of histogram sort (section 3.3: finish once every splitter has a
// probe in its target range).
//
// q is the number of buckets.  It equals p except in a stage of multi-stage
// HSS (section 5.3), where q groups of processors take one bucket each: the
// splitters are then i = 1..q-1 with ideal ranks N i/q, and every formula of
// sections 2 and 4.2 that counts buckets uses q (READING: the tolerance
// N eps/(2q), the final ratio 2 ln q / eps and the rate q s_j / N), while the
// histogram still runs over the p segments.
void determine_splitters(const Problem& P, uint32_t q, double eps, uint64_t seed,
                         uint32_t k_override, uint32_t max_rounds, int force_full,
                         uint32_t budget, int picks_mode, int trace_level, int threads, Run& R) {
    const uint64_t n = P.n;
    const uint32_t p = P.p;
    R.c = make_constants(n, q, eps, k_override);
    const uint64_t tol = R.c.tol;

    std::vector<Splitter> sp(q + 1);    // index 1..q-1
    std::vector<uint64_t> ideal(q + 1);
    for (uint32_t i = 0; i <= q; ++i) ideal[i] = ideal_rank(n, q, i);

    uint32_t unsettled = q - 1;
    for (uint32_t j = 1; unsettled > 0; ++j) {
        if (max_rounds && j > max_rounds) { R.status = -5; return; }
        RoundTrace tr;

        // Step 4 (sampling phase): the domain gamma_{j-1} is the union of the
        // open splitter intervals (L_i, U_i) of the splitters still unsettled
        // (READING: settled splitters are frozen, the interval end points are
        // already probes).  Identical intervals are taken once.
        std::map<std::pair<uint64_t, uint64_t>, bool> intervals;   // (L tag, U tag)
        for (uint32_t i = 1; i < q; ++i)
            if (!sp[i].settled) intervals[{sp[i].L, sp[i].U}] = true;
        std::vector<std::pair<uint64_t, uint64_t>> ivl(intervals.size());
        {
            size_t k = 0;
            for (auto& kv : intervals) ivl[k++] = kv.first;
        }
        // slice [lo, hi) of every segment inside every interval, at
        // slices[k p + s]; each processor finds the slices of its segment
        std::vector<std::pair<uint64_t, uint64_t>> slices(ivl.size() * p);
        std::vector<uint64_t> dom_part(threads < 1 ? 1 : threads, 0);
        split_over(p, threads, [&](int t, uint64_t s0, uint64_t s1) {
            for (uint64_t s = s0; s < s1; ++s) {
                for (size_t k = 0; k < ivl.size(); ++k) {
                    uint64_t Lg = ivl[k].first, Ug = ivl[k].second;
                    uint64_t lo = 0, hi = P.seg_len((uint32_t)s);
                    if (Lg != NONE) lo = P.count_below((uint32_t)s, Lg) + (P.segment_of(Lg) == s ? 1 : 0);
                    if (Ug != NONE) hi = P.count_below((uint32_t)s, Ug);
                    slices[k * p + s] = {P.seg_start[s] + lo, P.seg_start[s] + std::max(lo, hi)};
                    dom_part[t] += hi > lo ? hi - lo : 0;
                }
            }
        });
        for (uint64_t d : dom_part) tr.domain += d;

        uint32_t thresh;
        uint64_t max_seg = 0;
        for (uint32_t s = 0; s < p; ++s) max_seg = std::max(max_seg, P.seg_len(s));
        bool all = picks_mode ? pick_count(n, max_seg, tr.domain, budget, &thresh)
                   : budget   ? budget_threshold(tr.domain, q, budget, &thresh)
                              : sampling_threshold(n, q, R.c, j, &thresh);
        if (force_full) all = true;
        tr.thresh = all ? 0xFFFFFFFFu : thresh;
        tr.all = all ? 1u : 0u;

        // Section 4.2.1: each key of the domain is taken independently with
        // the round's probability.
        // Every processor draws for the keys of its own segment.
        std::vector<std::vector<uint64_t>> drawn(threads < 1 ? 1 : threads);
        if (picks_mode && !all) {
            // section 6: thresh picks of the whole segment, those inside an
            // interval's slice kept, each position once
            split_over(p, threads, [&](int t, uint64_t s0, uint64_t s1) {
                for (uint64_t s = s0; s < s1; ++s) {
                    std::vector<std::pair<uint64_t, uint64_t>> mine;   // the segment's slices
                    for (size_t k = 0; k < ivl.size(); ++k)
                        if (slices[k * p + s].second > slices[k * p + s].first) mine.push_back(slices[k * p + s]);
                    std::sort(mine.begin(), mine.end());
                    std::vector<uint64_t> kept;
                    for (uint32_t l = 0; l < thresh; ++l) {
                        const uint64_t g = P.seg_start[s] + pick_position(seed, l, (uint32_t)s, j, P.seg_len((uint32_t)s));
                        // the last slice starting at or before g
                        auto it = std::upper_bound(mine.begin(), mine.end(), std::make_pair(g, ~(uint64_t)0));
                        if (it != mine.begin() && g < std::prev(it)->second) kept.push_back(g);
                    }
                    std::sort(kept.begin(), kept.end());
                    kept.erase(std::unique(kept.begin(), kept.end()), kept.end());
                    drawn[t].insert(drawn[t].end(), kept.begin(), kept.end());
                }
            });
        } else {
            split_over(p, threads, [&](int t, uint64_t s0, uint64_t s1) {
                for (uint64_t s = s0; s < s1; ++s)
                    for (size_t k = 0; k < ivl.size(); ++k) {
                        const auto& sl = slices[k * p + s];
                        for (uint64_t g = sl.first; g < sl.second; ++g)
                            if (all || philox_word(seed, g, j) < thresh) drawn[t].push_back(g);
                    }
            });
        }
        std::vector<uint64_t> probes;
        for (auto& d : drawn) probes.insert(probes.end(), d.begin(), d.end());

        // Gather and sort the probes (section 5.1), in the strict order.
        std::sort(probes.begin(), probes.end(),
                  [&](uint64_t x, uint64_t y) { return before(P, x, y); });

        // Step 2: histogram of the probes against every segment, summed over
        // the segments (the reduction) -> global rank R(e) of each probe.
        // Every processor counts its own segment (the local histogram); the
        // counts are then added up over the processors.
        const size_t m = probes.size();
        std::vector<uint64_t> rk(m, 0);
        if (trace_level >= 2) tr.counts.assign(m * p, 0);
        std::vector<std::vector<uint64_t>> part(threads < 1 ? 1 : threads);
        split_over(p, threads, [&](int t, uint64_t s0, uint64_t s1) {
            part[t].assign(m, 0);
            for (uint64_t s = s0; s < s1; ++s)
                for (size_t e = 0; e < m; ++e) {
                    uint64_t c = P.count_below((uint32_t)s, probes[e]);
                    if (trace_level >= 2) tr.counts[e * p + s] = (uint32_t)c;
                    part[t][e] += c;
                }
        });
        for (auto& pt : part)
            for (size_t e = 0; e < pt.size(); ++e) rk[e] += pt[e];

        // Step 3 and step 5: for every unsettled splitter, a probe whose rank
        // lies in the target range settles it (READING: the closest to Ni/p,
        // the lower rank on a tie); otherwise the bounds L and U move to the
        // closest probe ranks below and above Ni/p.
        for (uint32_t i = 1; i < q; ++i) {
            Splitter& S = sp[i];
            if (S.settled) continue;
            size_t best = SIZE_MAX;
            uint64_t best_d = 0;
            for (size_t e = 0; e < probes.size(); ++e) {
                uint64_t d = rk[e] >= ideal[i] ? rk[e] - ideal[i] : ideal[i] - rk[e];
                if (d > tol) continue;
                if (best == SIZE_MAX || d < best_d || (d == best_d && rk[e] < rk[best])) {
                    best = e; best_d = d;
                }
            }
            if (best != SIZE_MAX) {
                S.settled = true;
                S.chi = rk[best];
                S.S = probes[best];
                --unsettled;
                continue;
            }
            for (size_t e = 0; e < probes.size(); ++e) {
                if (rk[e] < ideal[i]) {
                    if (S.L == NONE || rk[e] > S.Lrank) { S.L = probes[e]; S.Lrank = rk[e]; }
                } else {
                    if (S.U == NONE || rk[e] < S.Urank) { S.U = probes[e]; S.Urank = rk[e]; }
                }
            }
        }

        if (trace_level >= 1) {
            tr.probe_tag = probes;
            for (uint64_t g : probes) tr.probe_key.push_back(P.key[g]);
            tr.probe_rank = rk;
            tr.lo_rank.resize(q - 1); tr.hi_rank.resize(q - 1);
            tr.settled.resize(q - 1); tr.chi.resize(q - 1);
            for (uint32_t i = 1; i < q; ++i) {
                tr.lo_rank[i - 1] = sp[i].settled || sp[i].L == NONE ? NONE : sp[i].Lrank;
                tr.hi_rank[i - 1] = sp[i].settled || sp[i].U == NONE ? NONE : sp[i].Urank;
                tr.settled[i - 1] = sp[i].settled ? 1 : 0;
                tr.chi[i - 1] = sp[i].settled ? sp[i].chi : 0;
            }
        } else {
            tr.probe_rank.assign(rk.size(), 0);   // keeps m_j without the full trace
        }
        R.rounds.push_back(std::move(tr));
    }

    // Splitter ranks chi(0) = 0, chi(q) = N, and the piece boundaries c_s(S(b)).
    R.chi.assign(q + 1, 0);
    R.S_key.assign(q + 1, 0);
    R.S_tag.assign(q + 1, NONE);
    R.chi[q] = n;
    R.pieces.assign((size_t)(q + 1) * p, 0);
    for (uint32_t s = 0; s < p; ++s) R.pieces[(size_t)q * p + s] = P.seg_len(s);
    for (uint32_t i = 1; i < q; ++i) {
        R.chi[i] = sp[i].chi;
        R.S_tag[i] = sp[i].S;
        R.S_key[i] = P.key[sp[i].S];
    }
    split_over(p, threads, [&](int, uint64_t s0, uint64_t s1) {
        for (uint64_t s = s0; s < s1; ++s)
            for (uint32_t i = 1; i < q; ++i)
                R.pieces[(size_t)i * p + s] = P.count_below((uint32_t)s, sp[i].S);
    });
}

}  // namespace

extern "C" {

// Full HSS on the host.  mode 0 = partition (bucket b holds the keys of ranks
// [chi(b), chi(b+1)), pieces in ascending segment order, each in local sorted
// order), mode 1 = sort (each bucket additionally sorted stably by key).
// q = 0 means q = p buckets; 1 <= q <= p otherwise (one stage of multi-stage
// HSS, section 5.3: offsets_out then holds q+1 words).
// Returns a run handle (never NULL); oracle_status() tells the outcome.
oracle_run* oracle_hss(uint64_t n, uint32_t p, uint32_t q, double eps, int key_bits,
                       const void* keys_in, const uint64_t* vals_in, uint64_t seed,
                       int mode, uint32_t k_override, uint32_t max_rounds, int force_full,
                       uint32_t probes_per_round, int trace_level, void* keys_out,
                       uint64_t* vals_out, uint64_t* offsets_out, int threads, int picks_mode) {
    Run* R = new Run();
    if (q == 0) q = p;
    if (!valid_params(n, p, eps, key_bits) || q > p || !keys_in || !keys_out || !offsets_out ||
        (picks_mode && probes_per_round == 0)) {
        R->status = -1;
        return (oracle_run*)R;
    }
    auto t0 = std::chrono::steady_clock::now();
    Problem P;
    load_and_local_sort(P, n, p, key_bits, keys_in, vals_in, threads);
    R->t_local = seconds_since(t0);
    t0 = std::chrono::steady_clock::now();
    determine_splitters(P, q, eps, seed, k_override, max_rounds, force_full, probes_per_round,
                        picks_mode, trace_level, threads, *R);
    R->t_rounds = seconds_since(t0);
    if (R->status != 0) return (oracle_run*)R;

    // Data exchange (section 3.1 step 3): bucket b gathers, from every
    // segment in turn, the keys ranked in [chi(b), chi(b+1)).  Every
    // destination processor receives its own bucket.
    t0 = std::chrono::steady_clock::now();
    std::vector<uint64_t> ok(n), ov(n);
    std::vector<int> bad(q, 0);
    split_over(q, threads, [&](int, uint64_t b0, uint64_t b1) {
        for (uint64_t b = b0; b < b1; ++b) {
            uint64_t total = 0;
            for (uint32_t s = 0; s < p; ++s)
                total += R->pieces[(size_t)(b + 1) * p + s] - R->pieces[(size_t)b * p + s];
            if (total != R->chi[b + 1] - R->chi[b]) { bad[b] = 1; continue; }
            uint64_t o = R->chi[b];
            for (uint32_t s = 0; s < p; ++s) {
                uint64_t from = P.seg_start[s] + R->pieces[(size_t)b * p + s];
                uint64_t to = P.seg_start[s] + R->pieces[(size_t)(b + 1) * p + s];
                for (uint64_t g = from; g < to; ++g) { ok[o] = P.key[g]; ov[o] = P.val[g]; ++o; }
            }
        }
    });
    for (int x : bad)
        if (x) { R->status = -4; return (oracle_run*)R; }
    R->t_exchange = seconds_since(t0);
    // Local merge after the exchange (section 5): a stable sort of the bucket,
    // by every destination processor.
    t0 = std::chrono::steady_clock::now();
    if (mode == 1) {
        split_over(q, threads, [&](int, uint64_t b0, uint64_t b1) {
            for (uint64_t b = b0; b < b1; ++b) {
                uint64_t lo = R->chi[b], hi = R->chi[b + 1];
                std::vector<uint64_t> idx(hi - lo);
                std::iota(idx.begin(), idx.end(), lo);
                std::stable_sort(idx.begin(), idx.end(),
                                 [&](uint64_t x, uint64_t y) { return ok[x] < ok[y]; });
                std::vector<uint64_t> k2(hi - lo), v2(hi - lo);
                for (uint64_t t = 0; t < hi - lo; ++t) { k2[t] = ok[idx[t]]; v2[t] = ov[idx[t]]; }
                std::copy(k2.begin(), k2.end(), ok.begin() + lo);
                std::copy(v2.begin(), v2.end(), ov.begin() + lo);
            }
        });
    }
    R->t_final = seconds_since(t0);
    split_over(q, threads, [&](int, uint64_t b0, uint64_t b1) {
        for (uint64_t i = R->chi[b0]; i < R->chi[b1]; ++i) {
            if (key_bits == 32) ((uint32_t*)keys_out)[i] = (uint32_t)ok[i];
            else ((uint64_t*)keys_out)[i] = ok[i];
            if (vals_out) vals_out[i] = ov[i];
        }
    });
    for (uint32_t b = 0; b <= q; ++b) offsets_out[b] = R->chi[b];
    return (oracle_run*)R;
}

// Seconds spent per stage by the run: local sort, splitter rounds, exchange,
// bucket sort (mode 1; 0 otherwise).
void oracle_times(const oracle_run* h, double* out) {
    const Run* R = (const Run*)h;
    out[0] = R->t_local;
    out[1] = R->t_rounds;
    out[2] = R->t_exchange;
    out[3] = R->t_final;
}

// Local sort alone (section 6 phase 1).  Pinned: numpy's stable sort.
int oracle_local_sort(uint64_t n, uint32_t p, int key_bits, const void* keys_in,
                      const uint64_t* vals_in, void* keys_out, uint64_t* vals_out) {
    if (n == 0 || p == 0 || (uint64_t)p > n || (key_bits != 32 && key_bits != 64)) return -1;
    Problem P;
    load_and_local_sort(P, n, p, key_bits, keys_in, vals_in, 1);
    for (uint64_t i = 0; i < n; ++i) {
        if (key_bits == 32) ((uint32_t*)keys_out)[i] = (uint32_t)P.key[i];
        else ((uint64_t*)keys_out)[i] = P.key[i];
        if (vals_out) vals_out[i] = P.val[i];
    }
    return 0;
}

int oracle_status(const oracle_run* h) { return ((const Run*)h)->status; }
uint32_t oracle_num_rounds(const oracle_run* h) { return (uint32_t)((const Run*)h)->rounds.size(); }
uint64_t oracle_tol(const oracle_run* h) { return ((const Run*)h)->c.tol; }
uint32_t oracle_k(const oracle_run* h) { return ((const Run*)h)->c.k; }

// Per-round summary: domain size |gamma_{j-1}|, probe count m_j, threshold.
void oracle_round_info(const oracle_run* h, uint32_t j, uint64_t* domain, uint64_t* m,
                       uint32_t* thresh, uint32_t* all) {
    const RoundTrace& t = ((const Run*)h)->rounds[j];
    *domain = t.domain;
    *m = t.probe_rank.size();
    *thresh = t.thresh;
    *all = t.all;
}

// Per-round probes (sorted), their ranks, and (trace level 2) the count matrix.
void oracle_round_probes(const oracle_run* h, uint32_t j, uint64_t* keys, uint64_t* tags,
                         uint64_t* ranks, uint32_t* counts) {
    const RoundTrace& t = ((const Run*)h)->rounds[j];
    for (size_t e = 0; e < t.probe_rank.size(); ++e) {
        if (keys && e < t.probe_key.size()) keys[e] = t.probe_key[e];
        if (tags && e < t.probe_tag.size()) tags[e] = t.probe_tag[e];
        if (ranks) ranks[e] = t.probe_rank[e];
    }
    if (counts) std::copy(t.counts.begin(), t.counts.end(), counts);
}

// Per-round splitter state after the round (p-1 entries each).
void oracle_round_state(const oracle_run* h, uint32_t j, uint64_t* lo_rank, uint64_t* hi_rank,
                        uint8_t* settled, uint64_t* chi) {
    const RoundTrace& t = ((const Run*)h)->rounds[j];
    std::copy(t.lo_rank.begin(), t.lo_rank.end(), lo_rank);
    std::copy(t.hi_rank.begin(), t.hi_rank.end(), hi_rank);
    std::copy(t.settled.begin(), t.settled.end(), settled);
    std::copy(t.chi.begin(), t.chi.end(), chi);
}

// Final splitters: chi (p+1), S key and tag (p+1; entries 0 and p unused),
// and the piece matrix ((p+1) x p, row b = c_s(S(b))).
void oracle_splitters(const oracle_run* h, uint64_t* chi, uint64_t* s_key, uint64_t* s_tag,
                      uint64_t* pieces) {
    const Run* R = (const Run*)h;
    std::copy(R->chi.begin(), R->chi.end(), chi);
    if (s_key) std::copy(R->S_key.begin(), R->S_key.end(), s_key);
    if (s_tag) std::copy(R->S_tag.begin(), R->S_tag.end(), s_tag);
    if (pieces) std::copy(R->pieces.begin(), R->pieces.end(), pieces);
}

void oracle_free(oracle_run* h) { delete (Run*)h; }

}  // extern "C"
