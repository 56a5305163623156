// Prints rocRAND's Philox4x32-10 outputs (its public device/host API, run as a
// black box) for the (seed, subsequence, offset) triples given on stdin, one
// "seed sub offset" line each; output: four hex words per line.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        uint4 v = rocrand4(&st);
        std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
