// Host build of the count kernels' 128-bit helpers (paper_2404_11105_amd/csrc/u128.h)
// for tests/test_u128.py: the same inline functions the kernels call, compiled
// for the CPU so their carries can be compared with Python integers.
#include "../../paper_2404_11105_amd/csrc/u128.h"

extern "C" {

int t_u128_add(unsigned long long* lo, unsigned long long* hi, unsigned long long alo, unsigned long long ahi) {
    return xm::u128_add(*lo, *hi, alo, ahi) ? 1 : 0;
}

int t_u128_scale(unsigned long long* lo, unsigned long long* hi, uint32_t m) {
    return xm::u128_scale(*lo, *hi, m) ? 1 : 0;
}

// term value as (lo, hi) two's complement words; returns the overflow flag
int t_ie_term(int32_t coef, const uint32_t* h, uint32_t nb, unsigned long long* lo, unsigned long long* hi) {
    bool big = false;
    const __int128 v = xm::ie_term(coef, h, nb, &big);
    const unsigned __int128 u = (unsigned __int128)v;
    *lo = (unsigned long long)u;
    *hi = (unsigned long long)(u >> 64);
    return big ? 1 : 0;
}
}
