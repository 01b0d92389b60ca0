// Host-side driver for rocRAND's Philox4x32-10 block function, used only by the
// CPU test suite to cross-check the oracle's own Philox against an
// independently written library implementation.
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints the 4 output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// ten_rounds() is a protected member; a derived type exposes it.
struct Block : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Block eng;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.eval(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
