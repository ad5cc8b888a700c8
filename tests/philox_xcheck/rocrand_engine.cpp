// Prints Philox4x32-10 blocks from rocRAND's header engine (a third-party
// implementation used only to pin the oracle). Reads lines
// "seed subsequence offset" (offset in 32-bit words) and prints four words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
