// Prints rocRAND's Philox4x32-10 output words, used only to pin the oracle's
// own Philox implementation.  Reads lines "seed subsequence offset" from stdin
// and writes the next 32-bit word of rocRAND's philox4x32_10 engine placed at
// that (seed, subsequence, offset); with rocRAND's counter layout this is word
// (offset mod 4) of the block with counter (offset div 4, subsequence).
// Host code only: no GPU is touched.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        std::printf("%u\n", e.next());
    }
    return 0;
}
