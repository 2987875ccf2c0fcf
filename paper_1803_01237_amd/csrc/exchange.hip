// Data exchange of HSS on one device (section 3.1 step 3, section 5: the
// all-to-all becomes one bucketed scatter), for every instance of a plan.
//
// Piece (b, s) of an instance is the run [P(b, s), P(b+1, s)) of its locally
// sorted segment s, with P(b, s) = c_s(S(b)), P(0, s) = 0 and P(p, s) =
// |segment s|.  Bucket b receives its pieces in ascending s, starting at
// chi(b).  Buckets are numbered like segments (instance I's bucket b is
// seg0 + b).
//   offsets -- workgroup per bucket: exclusive scan of piece lengths over s,
//              checked against chi(b+1) - chi(b); copy workgroups per bucket
//   scan    -- one workgroup: first copy workgroup of every bucket
//   copy    -- workgroup per 4096 outputs of a bucket: the pieces that cover
//              them are staged in LDS; every output element finds its piece
//              by binary search there and copies one key (and payload);
//              consecutive lanes write consecutive outputs.

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kT = 256;
constexpr int kScanT = 1024;
constexpr int kChunk = 4096;
// LDS window of piece starts: at most kChunk non-empty pieces meet a chunk,
// but rarely more than a few hundred; a larger window would only cost
// occupancy (12 bytes per entry), so chunks meeting more pieces search the
// bucket's row in global memory instead
constexpr int kWindow = 1024;

__device__ __forceinline__ uint64_t piece_start(const ExchangeArgs& a, const InstDesc& D,
                                                uint32_t b, uint32_t s) {
    if (b == 0) return 0;
    if (b == D.q) return a.seg_off[D.seg0 + s + 1] - a.seg_off[D.seg0 + s];
    return a.prow[D.tab0 + (uint64_t)b * D.p + s];
}

// Rounds queued ahead of their read-back that did not settle every splitter
// (or overran a buffer): the exchange waits for the rounds that follow.
__device__ __forceinline__ bool gated(const ExchangeArgs& a) {
    return a.gate && (a.gate->n_after != 0 || a.gate->overflow != 0);
}

// Workgroup per row u = bucket b of its instance (the last row of an
// instance is none: no copy work).
__global__ __launch_bounds__(kT) void piece_offsets_kernel(ExchangeArgs a) {
    __shared__ uint64_t scratch[kT / kWave];
    if (gated(a)) return;
    const uint32_t u = blockIdx.x;
    const InstDesc D = a.inst[a.row_inst[u]];
    const uint32_t b = u - D.row0;
    if (b == D.q) {   // uniform over the workgroup
        if (threadIdx.x == 0) a.chunk0[u] = 0;
        return;
    }
    uint64_t run = 0;
    bool bad = false;
    for (uint32_t s0 = 0; s0 < D.p; s0 += kT) {
        const uint32_t s = s0 + threadIdx.x;
        uint64_t len = 0;
        if (s < D.p) {
            const uint64_t x0 = piece_start(a, D, b, s), x1 = piece_start(a, D, b + 1, s);
            if (x1 < x0) bad = true; else len = x1 - x0;
        }
        uint64_t tot;
        const uint64_t pre = block_exclusive_scan<uint64_t, kT>(len, scratch, &tot);
        if (s < D.p) a.dst[D.tab0 + (uint64_t)b * D.p + s] = (uint32_t)(run + pre);
        run += tot;
    }
    const uint64_t blen = a.chi_all[D.row0 + b + 1] - a.chi_all[D.row0 + b];
    const uint64_t max_bucket = (D.n + D.q - 1) / D.q + 2 * D.tol;
    if (bad || (threadIdx.x == 0 && (run != blen || blen > max_bucket)))
        atomicOr(a.err, kErrPieceSum);
    if (threadIdx.x == 0) a.chunk0[u] = (uint32_t)((min(blen, max_bucket) + kChunk - 1) / kChunk);
}

// One workgroup: exclusive scan of the copy workgroups per bucket.
__global__ __launch_bounds__(kScanT) void chunk_scan_kernel(ExchangeArgs a) {
    __shared__ uint64_t scratch[kScanT / kWave];
    if (gated(a)) return;
    const uint32_t n = a.n_rows;
    const uint32_t per = (n + kScanT - 1) / kScanT;
    const uint32_t r0 = min(threadIdx.x * per, n), r1 = min(r0 + per, n);
    uint64_t local = 0;
    for (uint32_t i = r0; i < r1; ++i) local += a.chunk0[i];
    uint64_t tot;
    uint64_t run = block_exclusive_scan<uint64_t, kScanT>(local, scratch, &tot);
    for (uint32_t i = r0; i < r1; ++i) {
        const uint64_t x = a.chunk0[i];
        a.chunk0[i] = (uint32_t)run;
        run += x;
    }
    if (threadIdx.x == 0) a.chunk0[n] = (uint32_t)tot;
}

// Last index in [lo, hi) of v with v[i] <= x (v[lo] <= x).
__device__ __forceinline__ uint32_t last_le_u32(const uint32_t* v, uint32_t lo, uint32_t hi,
                                                uint32_t x) {
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (v[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// The digit counts of a copy workgroup's outputs for the bucket sort (kCount).
template <typename K, bool kCount>
struct TileCount {
    uint32_t* hist = nullptr;   // LDS, 256 words
    K base = 0;
    int shift = 0;
    uint64_t am = ~0ull, om = 0;
    __device__ __forceinline__ void add(K k) {
        if constexpr (kCount) {
            const uint64_t x = (uint64_t)(K)(k - base);
            atomicAdd(&hist[(uint32_t)(x >> shift) & 0xFFu], 1u);
            am &= x;
            om |= x;
        }
    }
};

template <typename K, bool kPayload, bool kCount>
__global__ __launch_bounds__(kT) void exchange_copy_kernel(ExchangeArgs a, uint32_t window) {
    // window entries: piece start inside the bucket, source position of the piece
    extern __shared__ uint64_t smem[];
    uint64_t* w_src = smem;
    uint32_t* w_off = (uint32_t*)(smem + window);
    __shared__ uint32_t sh_first, sh_count;
    __shared__ uint32_t hist[kCount ? 256 : 1];
    __shared__ uint64_t red[kCount ? kT / kWave : 1][2];
    const uint32_t t = blockIdx.x;
    if (gated(a) || t >= a.chunk0[a.n_rows]) return;
    const uint32_t u = last_le_u32(a.chunk0, 0, a.n_rows, t);
    const InstDesc D = a.inst[a.row_inst[u]];
    const uint32_t b = u - D.row0;
    const uint64_t bstart = a.chi_all[D.row0 + b];
    const uint64_t blen = a.chi_all[D.row0 + b + 1] - bstart;
    const uint64_t r0 = (uint64_t)(t - a.chunk0[u]) * kChunk;
    // a consistent state has bstart + blen <= n; the bounds only keep an
    // inconsistent one (reported through err) inside the instance
    if (r0 >= blen || bstart + r0 >= D.n) return;
    const uint32_t r1 = (uint32_t)min(min(blen, r0 + kChunk), D.n - bstart);
    const uint32_t* row = a.dst + D.tab0 + (uint64_t)b * D.p;
    if (threadIdx.x == 0) {
        const uint32_t first = last_le_u32(row, 0, D.p, (uint32_t)r0);
        const uint32_t last = last_le_u32(row, first, D.p, r1 - 1);
        sh_first = first;
        sh_count = last - first + 1;
    }
    __syncthreads();
    const uint32_t first = sh_first, cnt = sh_count;
    const K* B = (const K*)a.B;
    K* out;
    uint64_t* vout;
    if (a.out) {
        out = (K*)a.out + D.pos0 + bstart;
        vout = kPayload ? a.vout + D.pos0 + bstart : nullptr;
    } else {
        const InstRun& R = a.run[a.row_inst[u]];
        out = (K*)R.kout + bstart;
        vout = kPayload ? R.vout + bstart : nullptr;
    }
    // a consistent state keeps every source inside its segment; the clamp only
    // keeps an inconsistent one (reported through err) inside the instance
    const uint64_t src_max = D.pos0 + D.n - 1;
    TileCount<K, kCount> tc;
    if constexpr (kCount) {
        tc.hist = hist;
        tc.base = (K)a.sort_base[b];
        tc.shift = a.sort_shift[b];
        hist[threadIdx.x] = 0;   // kT == 256
    }
    if (cnt > window) {
        // many empty pieces in the window: search the bucket's row directly
        if constexpr (kCount) __syncthreads();
        for (uint32_t r = (uint32_t)r0 + threadIdx.x; r < r1; r += kT) {
            const uint32_t s = last_le_u32(row, first, first + cnt, r);
            const uint64_t src = min(a.seg_off[D.seg0 + s] + piece_start(a, D, b, s) + (r - row[s]), src_max);
            const K k = B[src];
            out[r] = k;
            tc.add(k);
            if constexpr (kPayload) vout[r] = a.Bv[src];
        }
    } else {
        for (uint32_t i = threadIdx.x; i < cnt; i += kT) {
            const uint32_t s = first + i;
            w_off[i] = row[s];
            w_src[i] = a.seg_off[D.seg0 + s] + piece_start(a, D, b, s);
        }
        __syncthreads();
        // kG keys a thread at a time: their sources first, then all their
        // loads in flight together, then the stores (the loads of one key
        // after another waited out each one's latency; all of a thread's
        // keys at once cost occupancy)
        constexpr int kG = 4;
        for (uint32_t rb = (uint32_t)r0 + threadIdx.x; rb < r1; rb += kG * kT) {
            uint64_t src[kG];
#pragma unroll
            for (int q = 0; q < kG; ++q) {
                const uint32_t r = rb + (uint32_t)q * kT;
                src[q] = 0;
                if (r < r1) {
                    const uint32_t j = last_le_u32(w_off, 0, cnt, r);
                    src[q] = min(w_src[j] + (r - w_off[j]), src_max);
                }
            }
            K kv[kG];
            uint64_t vv[kPayload ? kG : 1];
#pragma unroll
            for (int q = 0; q < kG; ++q) {
                const bool in = rb + (uint32_t)q * kT < r1;
                kv[q] = in ? as_global(B)[src[q]] : (K)0;
                if constexpr (kPayload) vv[q] = in ? as_global(a.Bv)[src[q]] : 0;
            }
#pragma unroll
            for (int q = 0; q < kG; ++q) {
                const uint32_t r = rb + (uint32_t)q * kT;
                if (r < r1) {
                    as_global(out)[r] = kv[q];
                    tc.add(kv[q]);
                    if constexpr (kPayload) as_global(vout)[r] = vv[q];
                }
            }
        }
    }
    if constexpr (kCount) {
        // this workgroup's outputs are tile r0 / 4096 of bucket b
        uint64_t am = tc.am, om = tc.om;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            am &= shfl_u64(am, (int)(lane_id() ^ (uint32_t)o));
            om |= shfl_u64(om, (int)(lane_id() ^ (uint32_t)o));
        }
        if (lane_id() == 0) {
            red[threadIdx.x / kWave][0] = am;
            red[threadIdx.x / kWave][1] = om;
        }
        __syncthreads();
        const uint64_t tile = (uint64_t)b * a.sort_tps + r0 / kChunk;
        a.sort_counts[tile * 256 + threadIdx.x] = hist[threadIdx.x];
        if (threadIdx.x == 0) {
#pragma unroll
            for (int q = 1; q < kT / kWave; ++q) {
                am &= red[q][0];
                om |= red[q][1];
            }
            atomicAnd((unsigned long long*)&a.sort_and[b], (unsigned long long)am);
            atomicOr((unsigned long long*)&a.sort_or[b], (unsigned long long)om);
        }
    }
}

__global__ void bucket_shift_kernel(uint32_t p, int key_bits, const uint64_t* __restrict__ s_key,
                                    uint8_t* __restrict__ shift, uint64_t* __restrict__ base) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p) return;
    const uint64_t top = key_bits == 64 ? ~0ull : 0xFFFFFFFFull;
    const uint64_t lo = b == 0 ? 0 : s_key[b];
    const uint64_t hi = b + 1 == p ? top : s_key[b + 1];
    const uint64_t w = hi - lo;                           // offsets lie in [0, w]
    const int len = w ? 64 - __clzll((long long)w) : 0;   // bits of w
    shift[b] = (uint8_t)(len > 8 ? len - 8 : 0);
    base[b] = lo;
}

}  // namespace

hipError_t launch_bucket_shift(uint32_t p, int key_bits, const uint64_t* s_key, uint8_t* shift,
                               uint64_t* base, hipStream_t s) {
    hipLaunchKernelGGL(bucket_shift_kernel, dim3((p + 255) / 256), dim3(256), 0, s, p, key_bits,
                       s_key, shift, base);
    return hipGetLastError();
}

uint64_t exchange_chunk_bound(uint64_t total, uint32_t buckets) {
    return total / kChunk + buckets + 1;
}

// Offsets of two-stage HSS: final bucket g (p/r) + i starts where bucket i
// of group g starts inside the group, shifted by the group's start.
__global__ void stage_offsets_kernel(const uint64_t* chi1, const uint64_t* off2, uint32_t r,
                                     uint32_t pg, uint64_t n, uint64_t* out) {
    const uint64_t total = (uint64_t)r * pg;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        if (x == total) {
            out[x] = n;
            continue;
        }
        const uint64_t g = x / pg, i = x - g * pg;
        out[x] = chi1[g] + off2[g * (pg + 1) + i];
    }
}

__global__ void entry_ranges_kernel(uint32_t n_msd, const uint32_t* __restrict__ msd_seg,
                                    const uint32_t* __restrict__ seg_inst,
                                    const uint8_t* __restrict__ ishift, const uint64_t* __restrict__ ibase,
                                    uint8_t* __restrict__ shift, uint64_t* __restrict__ base) {
    for (uint32_t li = blockIdx.x * blockDim.x + threadIdx.x; li < n_msd; li += gridDim.x * blockDim.x) {
        const uint32_t I = seg_inst[msd_seg[li]];
        shift[li] = ishift[I];
        base[li] = ibase[I];
    }
}

hipError_t launch_entry_ranges(uint32_t n_msd, const uint32_t* msd_seg, const uint32_t* seg_inst,
                               const uint8_t* ishift, const uint64_t* ibase, uint8_t* shift,
                               uint64_t* base, hipStream_t s) {
    if (n_msd == 0) return hipSuccess;
    const uint32_t grid = std::min<uint32_t>((n_msd + kT - 1) / kT, 1024);
    hipLaunchKernelGGL(entry_ranges_kernel, dim3(grid), dim3(kT), 0, s, n_msd, msd_seg, seg_inst, ishift,
                       ibase, shift, base);
    return hipGetLastError();
}

hipError_t launch_stage_offsets(const uint64_t* chi1, const uint64_t* off2, uint32_t r, uint32_t pg,
                                uint64_t n, uint64_t* out, hipStream_t s) {
    const uint64_t total = (uint64_t)r * pg + 1;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((total + kT - 1) / kT, 1024);
    hipLaunchKernelGGL(stage_offsets_kernel, dim3(grid), dim3(kT), 0, s, chi1, off2, r, pg, n, out);
    return hipGetLastError();
}

hipError_t launch_exchange(const ExchangeArgs& a, hipStream_t s) {
    Profiler dummy;
    Profiler& prof = a.prof ? *a.prof : dummy;
    if (a.n_rows == 0) return hipSuccess;
    prof.begin(s);
    hipLaunchKernelGGL(piece_offsets_kernel, dim3(a.n_rows), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(chunk_scan_kernel, dim3(1), dim3(kScanT), 0, s, a);
    prof.end(kProfExchangeOffsets, s, 0);
    const dim3 grid((unsigned)a.max_chunks);
    const bool pay = a.Bv != nullptr;
    // LDS window: the pieces meeting one chunk, at most p entries and at most kWindow
    const uint32_t window = a.p_max < (uint32_t)kWindow ? a.p_max : (uint32_t)kWindow;
    const size_t lds = (size_t)window * (8 + 4);
    // algorithmic bytes: every key (and payload word) read once and written once
    prof.begin(s);
    const bool cnt = a.sort_counts != nullptr;
    if (a.key_bytes == 4) {
        if (cnt) {
            if (pay) hipLaunchKernelGGL((exchange_copy_kernel<uint32_t, true, true>), grid, dim3(kT), lds, s, a, window);
            else hipLaunchKernelGGL((exchange_copy_kernel<uint32_t, false, true>), grid, dim3(kT), lds, s, a, window);
        } else {
            if (pay) hipLaunchKernelGGL((exchange_copy_kernel<uint32_t, true, false>), grid, dim3(kT), lds, s, a, window);
            else hipLaunchKernelGGL((exchange_copy_kernel<uint32_t, false, false>), grid, dim3(kT), lds, s, a, window);
        }
    } else {
        if (cnt) {
            if (pay) hipLaunchKernelGGL((exchange_copy_kernel<uint64_t, true, true>), grid, dim3(kT), lds, s, a, window);
            else hipLaunchKernelGGL((exchange_copy_kernel<uint64_t, false, true>), grid, dim3(kT), lds, s, a, window);
        } else {
            if (pay) hipLaunchKernelGGL((exchange_copy_kernel<uint64_t, true, false>), grid, dim3(kT), lds, s, a, window);
            else hipLaunchKernelGGL((exchange_copy_kernel<uint64_t, false, false>), grid, dim3(kT), lds, s, a, window);
        }
    }
    prof.end(kProfExchangeCopy, s, a.total * 2 * (a.key_bytes + (pay ? 8 : 0)));
    return hipGetLastError();
}

}  // namespace hss
