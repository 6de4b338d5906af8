// Host-side probe: evaluates rocRAND's Philox4x32-10 engine at a given
// (counter, key), to cross-check the oracle's own Philox against a library
// implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) from stdin and prints
// the four output words (hex).  Runs on the CPU only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        unsigned long long sub = ((unsigned long long)c[3] << 32) | c[2];
        unsigned long long pos = ((unsigned long long)c[1] << 32) | c[0];
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        // discard(4a) advances the 64-bit block counter by a; step in pieces
        // of at most 2^61 blocks so that 4a never overflows.
        while (pos > 0) {
            unsigned long long a = pos < (1ull << 61) ? pos : (1ull << 61);
            e.discard(4ull * a);
            pos -= a;
        }
        unsigned a = e.next(), b = e.next(), d = e.next(), f = e.next();
        std::printf("%08x %08x %08x %08x\n", a, b, d, f);
    }
    return 0;
}
