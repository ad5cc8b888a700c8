// Prints Philox4x32-10 blocks from PyTorch's header-only engine (a third-party
// implementation used only to pin the oracle). Reads lines
// "seed subsequence offset" and prints the four 32-bit words of that block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        at::philox_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
