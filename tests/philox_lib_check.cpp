// Prints Philox4x32-10 blocks computed by PyTorch's header-only
// at::philox_engine, for cross-checking an independent implementation.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) from stdin and writes
// "x0 x1 x2 x3" for each.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>
#include <cstdio>

int main() {
    unsigned long long c[4], k[2];
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        // at::philox_engine(seed, subsequence, offset): key = seed (low, high),
        // counter = (offset low, offset high, subsequence low, subsequence high).
        uint64_t seed = (uint64_t)k[0] | ((uint64_t)k[1] << 32);
        uint64_t offset = (uint64_t)c[0] | ((uint64_t)c[1] << 32);
        uint64_t subseq = (uint64_t)c[2] | ((uint64_t)c[3] << 32);
        at::philox_engine eng(seed, subseq, offset);
        uint32_t x0 = eng(), x1 = eng(), x2 = eng(), x3 = eng();
        std::printf("%u %u %u %u\n", x0, x1, x2, x3);
    }
    return 0;
}
