// C entry points over the sub-block mask helpers, for the CPU tests.
#include "mvf_masks.h"

extern "C" {
uint32_t t_subblock_bits(uint64_t b) { return mvf::subblock_bits(b); }
uint64_t t_subblock_box(const int* lo, const int* hi) { return mvf::subblock_box(lo, hi); }
uint64_t t_cell_mask(const uint64_t* m8)
{
    uint64_t M[2][2][2];
    for (int i = 0; i < 8; ++i) M[i >> 2][(i >> 1) & 1][i & 1] = m8[i];
    return mvf::cell_mask(M);
}
}
