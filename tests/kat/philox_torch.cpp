// Philox4x32-10 known answers from PyTorch's header-only engine
// (ATen/core/PhiloxRNGEngine.h).  Reads lines "key0 key1 c0 c1 c2 c3" (hex)
// and prints the four output words of each counter.  The engine's counter is
// (offset lo, offset hi, subsequence lo, subsequence hi) and its key is
// (seed lo, seed hi).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::philox_engine e(seed, sub, off);
        unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
