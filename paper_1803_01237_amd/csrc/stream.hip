// A plain streaming copy, the measured ceiling that the streaming kernels of
// the local sort and the exchange are held against: every lane moves 16-byte
// words, four in flight per step, the workgroups spread over the whole buffer
// with a grid stride.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hss.h"

namespace {

constexpr int kT = 256;
constexpr int kUnroll = 4;
typedef unsigned int v4u __attribute__((ext_vector_type(4)));   // one 16-byte word

template <bool kNontemporal>
__global__ __launch_bounds__(kT) void stream_copy_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                         uint64_t words) {
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < words; i += kUnroll * stride) {
        v4u v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if constexpr (kNontemporal) v[u] = __builtin_nontemporal_load(src + i + u * stride);
            else v[u] = src[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if constexpr (kNontemporal) __builtin_nontemporal_store(v[u], dst + i + u * stride);
            else dst[i + u * stride] = v[u];
        }
    }
    for (; i < words; i += stride) {
        if constexpr (kNontemporal) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
        else dst[i] = src[i];
    }
}

}  // namespace

extern "C" hss_status hss_stream_copy(void* dst, const void* src, size_t bytes, uint32_t workgroups,
                                      int nontemporal, void* stream) {
    if (!dst || !src || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15) || workgroups == 0 ||
        workgroups > 65536)
        return HSS_ERR_INVALID_ARG;
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (bytes && a < b + bytes && b < a + bytes) return HSS_ERR_INVALID_ARG;
    if (bytes == 0) return HSS_OK;
    const uint64_t words = bytes / 16;
    const hipStream_t s = (hipStream_t)stream;
    if (nontemporal)
        hipLaunchKernelGGL(stream_copy_kernel<true>, dim3(workgroups), dim3(kT), 0, s, (const v4u*)src,
                           (v4u*)dst, words);
    else
        hipLaunchKernelGGL(stream_copy_kernel<false>, dim3(workgroups), dim3(kT), 0, s, (const v4u*)src,
                           (v4u*)dst, words);
    return hipGetLastError() == hipSuccess ? HSS_OK : HSS_ERR_DEVICE;
}
