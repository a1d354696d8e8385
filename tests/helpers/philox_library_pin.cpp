// Library reference for the Philox4x32-10 pin: PyTorch's header-only
// at::philox_engine (ATen/core/PhiloxRNGEngine.h).  Its state maps onto the
// generator's four counter words as (offset_lo, offset_hi, subsequence_lo,
// subsequence_hi) and onto the two key words as (seed_lo, seed_hi); four
// consecutive draws return the four output words of one block.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin, prints "w0 w1 w2 w3".
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint64_t seed = (k1 << 32) | k0;
        uint64_t subseq = (c3 << 32) | c2;
        uint64_t offset = (c1 << 32) | c0;
        at::philox_engine eng(seed, subseq, offset);
        uint32_t w[4];
        for (int i = 0; i < 4; ++i) w[i] = eng();
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
