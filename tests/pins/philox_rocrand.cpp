// Independent Philox4x32-10 for pinning the oracle: rocRAND's header-only
// engine, compiled for the host.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal
// u32) from stdin and prints the four output words of each counter/key.
//
// rocRAND's engine keeps the counter as (x, y, z, w); seeding with
// seed = k0 | k1 << 32 and subsequence = c2 | c3 << 32 sets (z, w); skipping
// 4 * c0 numbers sets x, and skips of c1 * 2^34 numbers (taken in pieces that
// fit 64 bits) set y, which positions it exactly on counter (c0, c1, c2, c3).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = k0 | (k1 << 32);
        unsigned long long sub = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        for (int i = 0; i < 4; ++i) e.discard((c1 >> 2) << 34);
        e.discard((c1 & 3ull) << 34);
        e.discard(4ull * c0);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
