// u128.h — unsigned 128-bit count arithmetic shared by the count kernels.
//
// Counts are exact unsigned 128-bit integers kept as (lo, hi) uint64 pairs
// (the paper does not bound them: a 5-leaf out-star on a 10^5-degree hub
// already has ~10^25 embeddings).  Every routine here reports a result that
// does not fit instead of wrapping silently.  The functions are plain
// integer code, callable on the host as well, so that their carries can be
// checked against arbitrary-precision integers on the CPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xm {

// (lo, hi) += (alo, ahi); returns true when the sum passed 2^128 - 1.
__host__ __device__ inline bool u128_add(unsigned long long& lo, unsigned long long& hi, unsigned long long alo,
                                         unsigned long long ahi) {
    const unsigned long long nlo = lo + alo;
    const unsigned long long c = nlo < lo ? 1ull : 0ull;
    const unsigned long long h1 = hi + ahi;
    const bool o1 = h1 < hi;
    const unsigned long long h2 = h1 + c;
    const bool o2 = h2 < h1;
    lo = nlo;
    hi = h2;
    return o1 || o2;
}

// (lo, hi) *= m; returns true when the product passed 2^128 - 1 (the words
// then hold the product modulo 2^128).
__host__ __device__ inline bool u128_scale(unsigned long long& lo, unsigned long long& hi, uint32_t m) {
    const unsigned __int128 pl = (unsigned __int128)lo * m;
    const unsigned __int128 ph = (unsigned __int128)hi * m + (unsigned long long)(pl >> 64);
    lo = (unsigned long long)pl;
    hi = (unsigned long long)ph;
    return (ph >> 64) != 0;
}

// Number of significant bits of x (0 for x = 0).
__host__ __device__ inline uint32_t u64_bits(unsigned long long x) {
    return x ? 64u - (uint32_t)__builtin_clzll(x) : 0u;
}

// One inclusion-exclusion term coef * h[0] * ... * h[nb-1] of a leaf group's
// injective count, in signed 128-bit arithmetic.  *big is set when the
// magnitude could reach 2^120: then a sum of at most 96 such terms could
// leave the signed 128-bit range, and the caller reports an overflow.
__host__ __device__ inline __int128 ie_term(int32_t coef, const uint32_t* h, uint32_t nb, bool* big) {
    const unsigned long long ac = (unsigned long long)(coef < 0 ? -(int64_t)coef : (int64_t)coef);
    uint32_t bits = u64_bits(ac);
    unsigned __int128 mag = ac;  // unsigned: a product past the range wraps, it is never undefined
    bool zero = ac == 0;
    for (uint32_t b = 0; b < nb; b++) {
        bits += u64_bits(h[b]);
        zero = zero || h[b] == 0;
        mag *= h[b];
    }
    if (zero) return 0;
    if (bits > 120) *big = true;
    return coef < 0 ? -(__int128)mag : (__int128)mag;
}

}  // namespace xm
