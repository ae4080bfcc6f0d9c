// Reference Philox4x32-10 outputs from rocRAND's host-callable engine.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) from stdin and prints the
// first four outputs of an engine whose key is (k0, k1) and whose counter is
// (c0, c1, c2, c3): seed = k1:k0, subsequence = c3:c2, offset = 4 * (c1:c0).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = (k1 << 32) | k0;
        const unsigned long long subseq = (c3 << 32) | c2;
        const unsigned long long offset = ((c1 << 32) | c0) * 4ull;
        rocrand_device::philox4x32_10_engine eng(seed, subseq, offset);
        unsigned int w[4];
        for (int k = 0; k < 4; ++k) w[k] = eng.next();
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
