// Host-only helper: evaluates rocRAND's own Philox4x32-10 block function on
// (counter, key) pairs read from stdin, one "k0 k1 c0 c1 c2 c3" per line, and
// prints the four output words.  Used to pin the oracle's generator against
// an independent, installed implementation.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct exposed : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    exposed e;
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        uint4 r = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
