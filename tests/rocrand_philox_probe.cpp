// Prints Philox4x32-10 blocks computed by rocRAND's open-source device/host
// engine (rocrand_philox4x32_10.h), used as an external pin for the oracle's
// own Philox.  Reads lines "k0 k1 c0 c1 c2 c3" (decimal) on stdin and prints
// "x0 x1 x2 x3" per line.  Runs on the host only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        // seed = key; subsequence fills counter words 2,3; offset/4 fills 0,1
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (k1 << 32) | k0;
        unsigned long long subsequence = (c3 << 32) | c2;
        unsigned long long offset = ((c1 << 32) | c0) * 4ull;
        rocrand_init(seed, subsequence, offset, &st);
        uint4 v = rocrand4(&st);
        std::printf("%u %u %u %u\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
