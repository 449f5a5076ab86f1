// Test helper: evaluates Philox4x32-10 through rocRAND's own engine (an
// independent, library implementation of the same published generator) for
// counters and keys read from stdin, so the oracle's generator can be pinned
// against it.  Host-only: built with hipcc, never run on a GPU.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// ten_rounds is a protected member of the engine; a derived class exposes it.
struct engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
    engine eng;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr = {c0, c1, c2, c3};
        uint2 key = {k0, k1};
        uint4 r = eng.block(ctr, key);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
