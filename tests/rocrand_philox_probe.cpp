// Test-only probe: evaluates rocRAND's own Philox4x32-10 bijection (a third,
// independent implementation) on counters/keys read from stdin, one
// "c0 c1 c2 c3 k0 k1" line in hex per query.  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct probe : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    probe p;
    unsigned v[6];
    while (std::scanf("%x %x %x %x %x %x", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6) {
        uint4 o = p.eval(uint4{v[0], v[1], v[2], v[3]}, uint2{v[4], v[5]});
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
