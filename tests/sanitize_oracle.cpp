// Drives the CPU oracle through its C interface on small shapes, for a build
// with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitize.py):
// every mode, key width, payload choice, bucket count, trace level and thread
// count, checking the sort output's order and the offsets on the way.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../oracle/hss_oracle.cpp"

namespace {

uint64_t next(uint64_t& x) {   // xorshift64*
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return x * 0x2545F4914F6CDD1DULL;
}

int failures = 0;

void check(bool ok, const char* what, uint64_t n, uint32_t p) {
    if (!ok) {
        std::printf("FAIL %s n=%llu p=%u\n", what, (unsigned long long)n, p);
        ++failures;
    }
}

void run(uint64_t n, uint32_t p, uint32_t q, double eps, int bits, bool payload, int mode, int trace,
         int threads, uint32_t budget, uint64_t seed, int dups, int picks = 0) {
    uint64_t x = seed * 0x9E3779B97F4A7C15ULL + 1;
    std::vector<uint64_t> k64(n), vals(n);
    std::vector<uint32_t> k32(n);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t v = next(x);
        if (dups) v %= (uint64_t)dups;
        k64[i] = v;
        k32[i] = (uint32_t)(v >> 32) ^ (uint32_t)v;
        vals[i] = i;
    }
    const void* kin = bits == 32 ? (const void*)k32.data() : (const void*)k64.data();
    std::vector<uint64_t> ko64(n);
    std::vector<uint32_t> ko32(n);
    std::vector<uint64_t> vo(n), off((q ? q : p) + 1);
    void* kout = bits == 32 ? (void*)ko32.data() : (void*)ko64.data();
    oracle_run* h = oracle_hss(n, p, q, eps, bits, kin, payload ? vals.data() : nullptr, seed, mode, 0, 0, 0,
                               budget, trace, kout, payload ? vo.data() : nullptr, off.data(), threads, picks);
    const int st = oracle_status(h);
    check(st == 0, "status", n, p);
    if (st == 0) {
        const uint32_t qq = q ? q : p;
        check(off[0] == 0 && off[qq] == n, "offsets ends", n, p);
        for (uint32_t b = 0; b < qq; ++b) check(off[b] <= off[b + 1], "offsets order", n, p);
        if (mode == 1)
            for (uint64_t i = 1; i < n; ++i) {
                const uint64_t a = bits == 32 ? ko32[i - 1] : ko64[i - 1], b = bits == 32 ? ko32[i] : ko64[i];
                if (a > b) { check(false, "sorted", n, p); break; }
            }
        const uint32_t rounds = oracle_num_rounds(h);
        for (uint32_t j = 0; j < rounds; ++j) {
            uint64_t dom = 0, m = 0;
            uint32_t th = 0, all = 0;
            oracle_round_info(h, j, &dom, &m, &th, &all);
            std::vector<uint64_t> pk(m), pt(m), pr(m);
            std::vector<uint32_t> cnt(trace >= 2 ? m * p : 0);
            oracle_round_probes(h, j, pk.data(), pt.data(), pr.data(), trace >= 2 ? cnt.data() : nullptr);
            if (trace >= 1 && qq > 1) {
                std::vector<uint64_t> lo(qq - 1), hi(qq - 1), chi(qq - 1);
                std::vector<uint8_t> settled(qq - 1);
                oracle_round_state(h, j, lo.data(), hi.data(), settled.data(), chi.data());
            }
        }
        std::vector<uint64_t> chi(qq + 1), sk(qq + 1), stg(qq + 1), pieces((uint64_t)(qq + 1) * p);
        oracle_splitters(h, chi.data(), sk.data(), stg.data(), pieces.data());
        double t[4];
        oracle_times(h, t);
    }
    oracle_free(h);
}

}  // namespace

int main() {
    run(1, 1, 0, 0.5, 64, true, 1, 2, 1, 0, 1, 0);
    run(300, 300, 0, 0.5, 64, true, 0, 2, 3, 0, 2, 0);
    run(5000, 16, 0, 0.05, 64, false, 1, 2, 1, 0, 3, 0);
    run(5000, 16, 0, 0.05, 64, true, 0, 1, 4, 0, 4, 0);
    run(20000, 37, 0, 0.02, 32, true, 1, 2, 5, 0, 5, 0);
    run(20000, 64, 8, 0.05, 64, true, 0, 1, 2, 0, 6, 0);
    run(12345, 20, 0, 1e-6, 64, false, 0, 2, 3, 0, 7, 0);          // tol = 0
    run(20000, 32, 0, 0.05, 64, true, 1, 2, 4, 0, 8, 101);         // many duplicates
    run(20000, 25, 0, 0.05, 64, true, 0, 1, 2, 0, 9, 1);           // all equal
    run(50000, 50, 0, 0.05, 64, false, 0, 1, 3, 5, 10, 0);         // probe budget
    run(50000, 50, 0, 0.05, 64, true, 1, 2, 3, 5, 11, 0, 1);       // the picks of section 6
    run(30000, 64, 0, 0.02, 32, false, 0, 1, 2, 1, 12, 300, 1);    // picks, duplicates
    std::vector<uint64_t> k(1000), ko(1000), v(1000), vo(1000);
    uint64_t x = 77;
    for (auto& a : k) a = next(x);
    for (size_t i = 0; i < v.size(); ++i) v[i] = i;
    check(oracle_local_sort(1000, 7, 64, k.data(), v.data(), ko.data(), vo.data()) == 0, "local sort", 1000, 7);
    uint64_t tol = 0;
    uint32_t kk = 0, th[40], al[40];
    double a = 0;
    oracle_constants(1ull << 28, 1024, 0.02, 0, &tol, &kk, &a, 40, th, al);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    (void)oracle_philox_word(1, 2, 3);
    // invalid arguments: a handle with status -1, freed
    oracle_run* h = oracle_hss(10, 11, 0, 0.1, 64, k.data(), nullptr, 1, 0, 0, 0, 0, 0, 0, ko.data(), nullptr,
                               vo.data(), 1, 0);
    check(oracle_status(h) == -1, "invalid", 10, 11);
    oracle_free(h);
    std::printf(failures ? "oracle sanitize: %d failures\n" : "oracle sanitize: ok\n", failures);
    return failures ? 1 : 0;
}
