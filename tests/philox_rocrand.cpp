// Prints Philox4x32-10 outputs computed by rocRAND's header implementation
// for counters/keys read from stdin ("c0 c1 c2 c3 k0 k1" per line).
// Test infrastructure: an independent implementation to pin the oracle's.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    probe p;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 r = p.run(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
