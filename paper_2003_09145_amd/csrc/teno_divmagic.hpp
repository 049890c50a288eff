// Division by an invariant integer as a multiply and shift (T. Granlund and
// P. L. Montgomery, "Division by invariant integers using multiplication",
// PLDI 1994, Thm 4.2 with N = 31): for d >= 1, l = ceil(log2 d) and
// m = ceil(2^(31 + l) / d), m < 2^32 and floor(x / d) = (x m) >> (31 + l)
// for every 0 <= x < 2^31.  Host-only (plain C++), so that the constants can
// be checked without a GPU.
#pragma once

#include <stdint.h>

namespace teno {

struct DivMagic {
    uint32_t m, sh;
};

inline DivMagic div_magic(uint32_t d) {
    int l = 0;
    while ((1ull << l) < d) ++l;
    return {(uint32_t)(((1ull << (31 + l)) + d - 1) / d), (uint32_t)(31 + l)};
}

}  // namespace teno
