// Reads lines "k0 k1 c0 c1 c2 c3" (decimal uint32) on stdin and prints the four
// Philox4x32-10 output words of PyTorch's own engine (ATen's philox_engine,
// an implementation independent of the oracle) for that key and counter.
// The engine's key is the 64-bit seed (low word first); its counter words are
// (offset low, offset high, subsequence low, subsequence high).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::philox_engine eng(seed, subseq, offset);
        uint32_t w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
