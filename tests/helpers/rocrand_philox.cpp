// Evaluates rocRAND's Philox4x32-10 block function on (counter, key) pairs read
// from stdin ("c0 c1 c2 c3 k0 k1" in hex, one per line) and prints the four
// output words in hex. Used only as an independent library reference for the
// oracle's generator; it runs on the host.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    using philox4x32_10_engine::ten_rounds;
};

int main()
{
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
