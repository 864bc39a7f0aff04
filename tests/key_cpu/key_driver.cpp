// Host build of the detector's rank-key helpers (lk_key.h): prints, for a
// seeded sequence of keys, bit positions and digits, every helper's result,
// which tests/test_key_cpu.py checks against Python integers.
#define __host__
#define __device__
#define __forceinline__ inline
#include "lk_key.h"

#include <cstdio>
#include <cstdlib>

using namespace lkmi;

static unsigned long long state = 0;

// splitmix64 (Steele, Lea, Flood 2014)
static unsigned long long next_u64()
{
    unsigned long long z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int main(int argc, char **argv)
{
    const int n = argc > 1 ? std::atoi(argv[1]) : 20000;
    state = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1;
    for (int i = 0; i < n; ++i) {
        Key k{next_u64(), (uint32_t)next_u64()};
        Key q{next_u64(), (uint32_t)next_u64()};
        // half of the pairs share a leading run of bits, of any length
        if (i & 1) {
            const int keep = (int)(next_u64() % 97);
            const unsigned __int128 a = key_top(k), b = key_top(q);
            const unsigned __int128 m = keep == 0 ? (unsigned __int128)0 : ~(unsigned __int128)0 << (128 - keep);
            const unsigned __int128 c = (a & m) | (b & ~m);
            q = Key{(unsigned long long)(c >> 64), (uint32_t)(c >> 32)};
        }
        const int p = (int)(next_u64() % 96), pe = (int)(next_u64() % 97);
        const uint32_t v = (uint32_t)(next_u64() & 0xFFu);
        const Key w = key_with_digit(q, p, v);
        std::printf("%016llx %08x %016llx %08x %d %d %u %u %d %d %016llx %08x\n", k.hi, k.lo, q.hi, q.lo, p, pe, v,
                    key_digit(k, p), (int)key_prefix_eq(k, q, pe), (int)key_less(k, q), w.hi, w.lo);
    }
    return 0;
}
