// Drives the host-side paths of libhss that run without a GPU -- argument
// checks, shape limits, workspace estimates and the workspace limit, error
// reporting, the release of plans that failed half-way -- for a build whose
// host code carries AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitize.py).  On a host without a device every call that
// reaches the device fails with HSS_ERR_DEVICE, which is one of the paths.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "hss.h"

namespace {

int failures = 0;

void expect(hss_status got, hss_status want, const char* what) {
    if (got != want) {
        std::printf("FAIL %s: %d (%s), expected %d\n", what, (int)got, hss_last_error(), (int)want);
        ++failures;
    }
}

}  // namespace

int main() {
    hss_plan_t p = nullptr;
    hss_tuning t{};
    expect(hss_plan(&p, 0, 1, 0.1, HSS_U64, 0, nullptr), HSS_ERR_INVALID_ARG, "n = 0");
    expect(hss_plan(&p, 10, 11, 0.1, HSS_U64, 0, nullptr), HSS_ERR_INVALID_ARG, "p > n");
    expect(hss_plan(&p, 10, 2, 1.0, HSS_U64, 0, nullptr), HSS_ERR_INVALID_ARG, "eps = 1");
    expect(hss_plan(&p, 10, 2, 0.1, (hss_key_type)7, 0, nullptr), HSS_ERR_INVALID_ARG, "key type");
    t.reserved[0] = 1;
    expect(hss_plan(&p, 100, 2, 0.1, HSS_U64, 0, &t), HSS_ERR_INVALID_ARG, "reserved field");
    t.reserved[0] = 0;
    expect(hss_plan_buckets(&p, 100, 8, 9, 0.1, HSS_U64, 0, nullptr), HSS_ERR_INVALID_ARG, "q > p");
    expect(hss_plan(&p, 1ull << 32, 8, 0.1, HSS_U64, 0, nullptr), HSS_ERR_UNSUPPORTED, "n >= 2^32");
    // the workspace limit stops the plan before any device call
    t.workspace_limit_mib = 16;
    expect(hss_plan(&p, 1ull << 28, 1024, 0.02, HSS_U64, 0, &t), HSS_ERR_OUT_OF_MEMORY, "limit, u64");
    expect(hss_plan(&p, 1ull << 24, 4096, 0.05, HSS_U32, 1, &t), HSS_ERR_OUT_OF_MEMORY, "limit, u32 payload");
    hss_instance_shape sh[3] = {{1u << 20, 64, HSS_U64, 0.05}, {1u << 16, 16, HSS_U32, 0.05},
                                {1u << 22, 256, HSS_U64, 0.02}};
    hss_batch_t bt = nullptr;
    t.workspace_limit_mib = 1;   // below the smaller key type's engine too
    expect(hss_batch_plan(&bt, sh, 3, 0, &t), HSS_ERR_OUT_OF_MEMORY, "limit, batch");
    t.workspace_limit_mib = 0;
    sh[1].p = 0;
    expect(hss_batch_plan(&bt, sh, 3, 0, nullptr), HSS_ERR_INVALID_ARG, "batch shape");
    hss_staged_t sp = nullptr;
    expect(hss_staged_plan(&sp, 1000, 16, 3, 0.05, 0.05, HSS_U64, 0, nullptr), HSS_ERR_INVALID_ARG, "groups");
    // no device here: the plan fails at its first device call and is released
    expect(hss_plan(&p, 1u << 20, 16, 0.05, HSS_U64, 0, nullptr), HSS_ERR_DEVICE, "no device");
    if (p) { std::printf("FAIL plan handle set\n"); ++failures; }
    // fixed workspace: sizes and limits on the host
    for (uint32_t kb = 0; kb < 2; ++kb)
        for (int pay = 0; pay < 2; ++pay)
            for (uint32_t pp : {1u, 7u, 256u}) {
                size_t b = 0, c = 0;
                expect(hss_partition_static_bytes(1u << 20, pp, 0.02, (hss_key_type)kb, pay, &b, &c), HSS_OK,
                       "static bytes");
                if (!(b > 0 && b <= c)) { std::printf("FAIL static bytes %zu %zu\n", b, c); ++failures; }
            }
    size_t b = 0, c = 0;
    expect(hss_partition_static_bytes((1u << 20) + 1, 16, 0.02, HSS_U64, 0, &b, &c), HSS_ERR_UNSUPPORTED, "static n");
    const uintptr_t a = (uintptr_t)1 << 40;   // aligned, far-apart addresses, never dereferenced
    expect(hss_partition_static(1u << 20, 257, 0.05, HSS_U64, 1, (const void*)a, nullptr, (void*)(a + (1u << 30)),
                                nullptr, (uint64_t*)(a + (2ull << 30)), nullptr),
           HSS_ERR_UNSUPPORTED, "static p");
    expect(hss_partition_static(1000, 16, 0.05, HSS_U64, 1, (const void*)a, nullptr, (void*)(a + 8), nullptr,
                                (uint64_t*)(a + (2ull << 30)), nullptr),
           HSS_ERR_INVALID_ARG, "static overlap");
    expect(hss_partition(nullptr, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr), HSS_ERR_INVALID_ARG,
           "null plan");
    expect(hss_stream_copy((void*)(a + 16), (const void*)a, 100, 4, 0, nullptr), HSS_ERR_INVALID_ARG, "copy size");
    hss_request rq{};
    rq.n = 1000;
    rq.p = 10;
    rq.key_type = HSS_U64;
    rq.eps = 0.05;
    if (hss_server_footprint(&rq) == 0) { std::printf("FAIL footprint\n"); ++failures; }
    for (int s = 0; s >= -5; --s)
        if (!std::strlen(hss_status_string((hss_status)s))) { std::printf("FAIL status string\n"); ++failures; }
    hss_plan_destroy(nullptr);
    hss_batch_destroy(nullptr);
    hss_staged_destroy(nullptr);
    std::printf(failures ? "host sanitize: %d failures\n" : "host sanitize: ok\n", failures);
    return failures ? 1 : 0;
}
