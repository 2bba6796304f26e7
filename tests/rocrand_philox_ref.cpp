// Independent comparator for the oracle's Philox4x32-10: rocRAND's engine, run on
// the host.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output
// words.  The engine is positioned on counter (c0, c1, c2, c3) with key (k0, k1)
// through its public API: seed = k0 | k1 << 32, subsequence = c2 | c3 << 32, then
// the low 64 counter bits are advanced with discard() in chunks of 2^61 blocks of
// four outputs, so that no offset overflows.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_device::philox4x32_10_engine eng(k0 | (k1 << 32), c2 | (c3 << 32), 0);
        unsigned long long blocks = c0 | (c1 << 32);
        const unsigned long long chunk = 1ull << 61;
        while (blocks > 0) {
            unsigned long long b = blocks < chunk ? blocks : chunk;
            eng.discard(4ull * b);
            blocks -= b;
        }
        uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
