// Host-only helper for the oracle's Philox pin: exposes rocRAND's own
// Philox4x32-10 block function (an implementation independent of the
// oracle) and evaluates it on "c0 c1 c2 c3 k0 k1" lines read from stdin.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Rounds : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Rounds e;
    unsigned a, b, c, d, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
        uint4 r = e.eval(make_uint4(a, b, c, d), make_uint2(k0, k1));
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
