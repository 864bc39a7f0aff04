// Rank keys of detector candidates and the bit fields the selection works
// on.  Written for the device; a host test supplies the function attributes
// and checks every helper against plain big-integer arithmetic.
#pragma once
#include <cstdint>

namespace lkmi {

// The rank key of a candidate: 96 bits, R bits then the complemented raster
// index (larger = earlier), so the order is total.  Digits are 8-bit fields
// at any bit position p (0 = the most significant bit), read from the key
// aligned to the top of 128 bits.
struct Key {
    unsigned long long hi;   // bits of R (R > 0, so the bits order like R)
    uint32_t lo;             // complemented raster index
};

__host__ __device__ __forceinline__ bool key_less(Key a, Key b)
{
    return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

__host__ __device__ __forceinline__ unsigned __int128 key_top(Key k)
{
    return ((unsigned __int128)k.hi << 64) | ((unsigned __int128)k.lo << 32);
}

// bits [p, p + 8) of the key, 0 <= p < 96 (bits past the key read as 0)
__host__ __device__ __forceinline__ uint32_t key_digit(Key k, int p)
{
    return (uint32_t)((key_top(k) << p) >> 120);
}

// the leading p bits of k and q agree, 0 <= p <= 96
__host__ __device__ __forceinline__ bool key_prefix_eq(Key k, Key q, int p)
{
    return p == 0 || ((key_top(k) ^ key_top(q)) >> (128 - p)) == 0;
}

// q's leading p bits, then digit v, then zeros: the least key whose digit at
// p is v among those with q's leading p bits, 0 <= p < 96
__host__ __device__ __forceinline__ Key key_with_digit(Key q, int p, uint32_t v)
{
    unsigned __int128 t = key_top(q);
    t = p == 0 ? (unsigned __int128)0 : (t >> (128 - p)) << (128 - p);
    t |= (unsigned __int128)(v & 0xFFu) << (120 - p);
    return Key{(unsigned long long)(t >> 64), (uint32_t)(t >> 32)};
}

}  // namespace lkmi
