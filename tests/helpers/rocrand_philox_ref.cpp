// Reference Philox4x32-10 blocks from rocRAND's public device/host API
// (rocrand_init + rocrand4), used as a black box to pin the oracle's own
// Philox implementation.  Reads "seed subsequence offset" triples from stdin
// and prints the four 32-bit words of the block at that position.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
