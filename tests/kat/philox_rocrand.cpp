// Philox4x32-10 known answers from rocRAND's header (rocrand_philox4x32_10.h),
// host side only.  Reads lines "key0 key1 c0 c1 c2 c3" (hex, c1 < 2^30) and
// prints the four output words.  rocRAND's offset counts 32-bit outputs, four
// per counter value; its subsequence fills counter words 2 and 3.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
