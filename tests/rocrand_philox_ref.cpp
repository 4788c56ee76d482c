// Host-only reference: evaluates rocRAND's Philox4x32-10 engine at explicit
// (key, counter) pairs.  Reads lines "k0 k1 c0 c1 c2 c3" on stdin and prints
// the four 32-bit output words of each block.  Used only by the test suite to
// pin the oracle's Philox against an independent implementation.
#include <cstdio>
#include <rocrand/rocrand_kernel.h>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // Word offset 4 * (c0 + c1 * 2^32) can exceed 64 bits: advance in pieces.
        rocrand_init(seed, subseq, 0ull, &st);
        skipahead(4ull * (unsigned long long)c0, &st);
        for (int rep = 0; rep < 4; ++rep) skipahead((unsigned long long)c1 << 32, &st);
        unsigned w0 = rocrand(&st), w1 = rocrand(&st), w2 = rocrand(&st), w3 = rocrand(&st);
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
