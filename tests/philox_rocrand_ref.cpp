// Reference Philox4x32-10 outputs from rocRAND's header-only engine (an
// implementation independent of the oracle's), used by the oracle pins.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) on stdin and prints the
// four output words of ten rounds on counter (c0, c1, c2, c3) under key
// (k0, k1).  Host code only: the engine's member functions are host-callable.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

namespace {
// ten_rounds is a protected member of the engine; a derived type exposes it.
struct Philox : rocrand_device::philox4x32_10_engine {
    uint4 bijection(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}  // namespace

int main() {
    Philox eng;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c;
        c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k;
        k.x = k0; k.y = k1;
        const uint4 r = eng.bijection(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    // the engine's public path: seed s, subsequence q, offset 0 puts counter
    // (0, 0, q_lo, q_hi) under key (s_lo, s_hi); its first four words must be
    // the bijection of that counter
    rocrand_device::philox4x32_10_engine pub(0x0123456789abcdefULL, 0x00000005deadbeefULL, 0);
    unsigned w[4];
    for (unsigned &v : w) v = pub.next();
    std::printf("engine %u %u %u %u\n", w[0], w[1], w[2], w[3]);
    return 0;
}
