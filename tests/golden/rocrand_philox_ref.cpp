// Independent reference for the Philox4x32-10 generator: rocRAND's own engine, run on the
// host.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the four output words.
// The engine is positioned so that its first block is philox(counter=(c0,c1,c2,c3), key=(k0,k1)):
// the seed supplies the key, the subsequence index the high counter words, and skipping
// 4 N outputs (four per block, in four steps of N so the count cannot overflow) advances
// the low counter words by N.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long sub = (c3 << 32) | c2;
        unsigned long long nblk = (c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine e(seed, sub, 0ull);
        for (int i = 0; i < 4; ++i) e.discard(nblk);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
