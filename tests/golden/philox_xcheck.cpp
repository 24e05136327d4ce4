// Independent Philox4x32-10 for cross-checking the oracle: drives the rocRAND
// engine's own ten-round function (installed source header) on host.
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints "w0 w1 w2 w3" (hex).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main()
{
    Probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = p.run(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
