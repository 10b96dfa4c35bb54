// Independent Philox4x32-10 reference for the oracle pin: rocRAND's
// header-only engine.  Reads "c0 c1 c2 c3 k0 k1" (hex) per line on stdin and
// prints the four output words of one block for counter (c0..c3), key (k0, k1).
// The engine's state is (key = seed, counter = subsequence << 64 | offset / 4),
// so seed = k0 | k1 << 32, subsequence = c2 | c3 << 32, offset = 4 (c0 | c1 << 32).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
