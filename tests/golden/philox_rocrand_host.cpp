// Independent Philox4x32-10 reference for the oracle's pin test.
// Built for the host only (no device code) from rocRAND's header engine.
// Reads lines "k0 k1 c0 c1 c2 c3" (decimal 32-bit words) on stdin and prints
// the four output words of Philox4x32-10 at that key and counter.
//
// Mapping onto rocRAND's (seed, subsequence, offset) interface:
//   key      = seed (low word k0, high word k1)
//   (c2, c3) = subsequence (low, high)
//   (c0, c1) = counter offset, reached by four skipahead() calls of
//              c0 + 2^32 c1 numbers each (each counter step is 4 numbers).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(k0 | (k1 << 32), c2 | (c3 << 32), 0ULL, &st);
        unsigned long long delta = c0 | (c1 << 32);
        for (int t = 0; t < 4; ++t) skipahead(delta, &st);
        unsigned int w[4];
        for (int t = 0; t < 4; ++t) w[t] = rocrand(&st);
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
