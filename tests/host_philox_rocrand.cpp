// The Philox4x32-10 bijection of rocRAND's header-only engine, an
// implementation of Salmon, Moraes, Dror and Shaw (SC'11) independent of
// this project, built for the host for a CPU test of the oracle's
// generator: for each line "c0 c1 c2 c3 k0 k1" read from stdin, prints the
// four output words of ten rounds on counter (c0..c3) and key (k0, k1).
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

struct Bijection : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Bijection b;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const uint4 o = b.apply(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
