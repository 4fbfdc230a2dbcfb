// Independent Philox4x32-10 known-answer probe built on rocRAND's header-only
// host engine.  Used only by the tests to pin the oracle's own Philox.
// rocRAND's engine(seed, subsequence, offset) runs counter
// (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi) under key
// (seed lo, seed hi).  Reads lines "seed c0 c1 c2 c3" (hex) from stdin.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llx %x %x %x %x", &seed, &c0, &c1, &c2, &c3) == 5) {
        const unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        const unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        const uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
