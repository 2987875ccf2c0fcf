// Data exchange of HSS on one device (section 3.1 step 3, section 5: the
// all-to-all becomes one bucketed scatter).
//
// Piece (b, s) is the run [P(b, s), P(b+1, s)) of locally sorted segment s,
// with P(b, s) = c_s(S(b)), P(0, s) = 0 and P(p, s) = |segment s|.  Bucket b
// receives its pieces in ascending s, starting at chi(b).
//   offsets -- workgroup per bucket: exclusive scan of piece lengths over s,
//              checked against chi(b+1) - chi(b)
//   copy    -- workgroup per (bucket, chunk of 4096 outputs): the pieces that
//              cover the chunk are staged in LDS; every output element finds
//              its piece by binary search there and copies one key (and
//              payload); consecutive lanes write consecutive outputs.

#include "device.hpp"
#include "internal.hpp"

namespace hss {

namespace {

constexpr int kT = 256;
constexpr int kChunk = 4096;
constexpr int kWindow = kChunk + 1;    // at most kChunk non-empty pieces meet a chunk

__device__ __forceinline__ uint64_t piece_start(const ExchangeArgs& a, uint32_t b, uint32_t s) {
    if (b == 0) return 0;
    if (b == a.p) return a.seg_off[s + 1] - a.seg_off[s];
    return a.prow[(uint64_t)b * a.p + s];
}

__global__ __launch_bounds__(kT) void piece_offsets_kernel(ExchangeArgs a) {
    __shared__ uint64_t scratch[kT / kWave];
    const uint32_t b = blockIdx.x;
    uint64_t run = 0;
    bool bad = false;
    for (uint32_t s0 = 0; s0 < a.p; s0 += kT) {
        const uint32_t s = s0 + threadIdx.x;
        uint64_t len = 0;
        if (s < a.p) {
            const uint64_t x0 = piece_start(a, b, s), x1 = piece_start(a, b + 1, s);
            if (x1 < x0) bad = true; else len = x1 - x0;
        }
        uint64_t tot;
        const uint64_t pre = block_exclusive_scan<uint64_t, kT>(len, scratch, &tot);
        if (s < a.p) a.dst[(uint64_t)b * a.p + s] = (uint32_t)(run + pre);
        run += tot;
    }
    const uint64_t blen = a.chi[b + 1] - a.chi[b];
    if (bad || (threadIdx.x == 0 && (run != blen || blen > a.max_bucket)))
        atomicOr(a.err, kErrPieceSum);
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

template <typename K, bool kPayload>
__global__ __launch_bounds__(kT) void exchange_copy_kernel(ExchangeArgs a, uint32_t chunks,
                                                           uint32_t window) {
    // window entries: piece start inside the bucket, source position of the piece
    extern __shared__ uint64_t smem[];
    uint64_t* w_src = smem;
    uint32_t* w_off = (uint32_t*)(smem + window);
    __shared__ uint32_t sh_first, sh_count;
    const uint32_t b = blockIdx.x / chunks;
    const uint32_t c = blockIdx.x % chunks;
    const uint64_t bstart = a.chi[b];
    const uint64_t blen = a.chi[b + 1] - bstart;
    const uint64_t r0 = (uint64_t)c * kChunk;
    if (r0 >= blen) return;
    const uint32_t r1 = (uint32_t)min(blen, r0 + kChunk);
    const uint32_t* row = a.dst + (uint64_t)b * a.p;
    if (threadIdx.x == 0) {
        const uint32_t first = last_le_u32(row, 0, a.p, (uint32_t)r0);
        const uint32_t last = last_le_u32(row, first, a.p, r1 - 1);
        sh_first = first;
        sh_count = last - first + 1;
    }
    __syncthreads();
    const uint32_t first = sh_first, cnt = sh_count;
    const K* B = (const K*)a.B;
    K* out = (K*)a.out;
    if (cnt > window) {
        // many empty pieces in the window: search the bucket's row directly
        for (uint32_t r = (uint32_t)r0 + threadIdx.x; r < r1; r += kT) {
            const uint32_t s = last_le_u32(row, first, first + cnt, r);
            const uint64_t src = min(a.seg_off[s] + piece_start(a, b, s) + (r - row[s]), a.n - 1);
            if (bstart + r >= a.n) break;
            out[bstart + r] = B[src];
            if constexpr (kPayload) a.vout[bstart + r] = a.Bv[src];
        }
        return;
    }
    for (uint32_t i = threadIdx.x; i < cnt; i += kT) {
        const uint32_t s = first + i;
        w_off[i] = row[s];
        w_src[i] = a.seg_off[s] + piece_start(a, b, s);
    }
    __syncthreads();
    for (uint32_t r = (uint32_t)r0 + threadIdx.x; r < r1; r += kT) {
        const uint32_t j = last_le_u32(w_off, 0, cnt, r);
        // a consistent state keeps src inside segment s; the clamps only keep an
        // inconsistent one (reported through err) inside the buffers
        const uint64_t src = min(w_src[j] + (r - w_off[j]), a.n - 1);
        if (bstart + r >= a.n) break;
        out[bstart + r] = B[src];
        if constexpr (kPayload) a.vout[bstart + r] = a.Bv[src];
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

hipError_t launch_exchange(const ExchangeArgs& a, hipStream_t s) {
    Profiler dummy;
    Profiler& prof = a.prof ? *a.prof : dummy;
    const uint64_t pp = (uint64_t)a.p * a.p;
    prof.begin(s);
    hipLaunchKernelGGL(piece_offsets_kernel, dim3(a.p), dim3(kT), 0, s, a);
    prof.end(kProfExchangeOffsets, s, pp * 4 * 3);
    const uint32_t chunks = (uint32_t)((a.max_bucket + kChunk - 1) / kChunk);
    if (chunks == 0) return hipGetLastError();
    const dim3 grid((unsigned)((uint64_t)a.p * chunks));
    const bool pay = a.Bv != nullptr;
    // LDS window: the pieces meeting one chunk, at most p and at most kWindow
    const uint32_t window = a.p < (uint32_t)kWindow ? a.p : (uint32_t)kWindow;
    const size_t lds = (size_t)window * (8 + 4);
    // algorithmic bytes: every key (and payload word) read once and written once
    prof.begin(s);
    if (a.key_bytes == 4) {
        if (pay) hipLaunchKernelGGL((exchange_copy_kernel<uint32_t, true>), grid, dim3(kT), lds, s, a, chunks, window);
        else hipLaunchKernelGGL((exchange_copy_kernel<uint32_t, false>), grid, dim3(kT), lds, s, a, chunks, window);
    } else {
        if (pay) hipLaunchKernelGGL((exchange_copy_kernel<uint64_t, true>), grid, dim3(kT), lds, s, a, chunks, window);
        else hipLaunchKernelGGL((exchange_copy_kernel<uint64_t, false>), grid, dim3(kT), lds, s, a, chunks, window);
    }
    prof.end(kProfExchangeCopy, s, a.n * 2 * (a.key_bytes + (pay ? 8 : 0)));
    return hipGetLastError();
}

}  // namespace hss
