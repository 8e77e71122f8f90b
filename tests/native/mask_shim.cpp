// C entry points over the sub-block mask helpers, for the CPU tests.
#include "mvf_masks.h"

extern "C" {
uint32_t t_subblock_bits(uint64_t b) { return mvf::subblock_bits(b); }
uint64_t t_subblock_box(const int* lo, const int* hi) { return mvf::subblock_box(lo, hi); }
void t_grow_clear_box(uint64_t cm, int* lo, int* hi, const float* dir) { mvf::grow_clear_box(cm, lo, hi, dir); }
uint64_t t_cell_mask(const uint64_t* m8)
{
    uint64_t M[2][2][2];
    for (int i = 0; i < 8; ++i) M[i >> 2][(i >> 1) & 1][i & 1] = m8[i];
    return mvf::cell_mask(M);
}
}
