// Independent Philox4x32-10 for pinning the oracle: evaluates rocRAND's
// host-callable engine at given (counter, key) pairs.  rocRAND's state keys
// the generator with (seed lo, seed hi) and starts at counter
// (offset / 4 as a 64-bit value in words 0-1, subsequence in words 2-3);
// skipahead by 4n numbers advances that block counter by n.
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints the 4 output words.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdint>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subsequence, 4ull * c0, &st);
        // add c1 * 2^32 to the 64-bit block counter in four steps of
        // c1 * 2^30 blocks, each an offset below 2^64 numbers
        for (int q = 0; q < 4; ++q)
            skipahead((unsigned long long)c1 << 32, &st);
        uint4 v = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
