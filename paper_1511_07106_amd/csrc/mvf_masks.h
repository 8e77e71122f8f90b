// Bit operations on the per-brick sub-block masks (fmask, cmask): 64 bits,
// bit z2 * 16 + y2 * 4 + x2 for the 2x2x2 sub-block (x2, y2, z2) of an 8^3
// brick.  Plain inline functions, compiled into the HIP kernels and, for
// tests, by a host C++ compiler.
#pragma once
#include <stdint.h>

#ifndef MVF_HD
#if defined(__HIPCC__)
#define MVF_HD __host__ __device__ __forceinline__
#else
#define MVF_HD inline
#endif
#endif

namespace mvf {

// Sub-block flags of one pair of z-slices of a brick: b holds one bit per
// voxel column (bit 8 y + x); returns bit y2 * 4 + x2 set if a column of the
// 2x2 group (x2, y2) had its bit set.
MVF_HD uint32_t subblock_bits(uint64_t b)
{
    b |= b >> 1;                                   // pair x with x + 1
    b |= b >> 8;                                   // pair y with y + 1
    b &= 0x0055005500550055ull;                    // keep x, y even: bit 16 y2 + 2 x2
    b = (b | (b >> 1)) & 0x0033003300330033ull;    // -> bit 16 y2 + x2
    b = (b | (b >> 2)) & 0x000f000f000f000full;
    b = (b | (b >> 12)) & 0x000000ff000000ffull;   // -> bit 4 y2 + x2
    b = (b | (b >> 24)) & 0xffffull;
    return (uint32_t)b;
}

// Bits lo..hi of a nibble (0 <= lo, hi <= 3; empty when lo > hi).
MVF_HD uint32_t nibble_range(int lo, int hi)
{
    return (0xfu >> (3 - hi)) & (0xfu << lo);
}

// Mask of the sub-blocks [lo, hi] (per axis, 0..3) of a brick, built from
// 32-bit halves (z rows 0-1 and 2-3).
MVF_HD uint64_t subblock_box(const int lo[3], const int hi[3])
{
    const uint32_t m16 = (nibble_range(lo[0], hi[0]) * 0x1111u) & (0xffffu >> (4 * (3 - hi[1]))) &
                         (0xffffu << (4 * lo[1]));
    const uint32_t zm = nibble_range(lo[2], hi[2]);
    const uint32_t lo32 = ((zm & 1u) ? m16 : 0u) | ((zm & 2u) ? (m16 << 16) : 0u);
    const uint32_t hi32 = ((zm & 4u) ? m16 : 0u) | ((zm & 8u) ? (m16 << 16) : 0u);
    return ((uint64_t)hi32 << 32) | lo32;
}

// Occupancy, per x, y or z sub-block slice, of a mask (bit z*16 + y*4 + x).
MVF_HD uint32_t occupancy_x(uint64_t m)
{
    uint32_t t = (uint32_t)m | (uint32_t)(m >> 32);
    t |= t >> 16;
    t |= t >> 8;
    t |= t >> 4;
    return t & 0xfu;
}
MVF_HD uint32_t occupancy_y(uint64_t m)
{
    uint32_t t = (uint32_t)m | (uint32_t)(m >> 32);
    t |= t >> 16;
    t |= t >> 1;
    t |= t >> 2;   // bit 4y: some x of row y
    return (t & 1u) | ((t >> 3) & 2u) | ((t >> 6) & 4u) | ((t >> 9) & 8u);
}
MVF_HD uint32_t occupancy_z(uint64_t m)
{
    return ((m & 0xffffull) ? 1u : 0u) | ((m & 0xffff0000ull) ? 2u : 0u) | ((m & 0xffff00000000ull) ? 4u : 0u) |
           ((m >> 48) ? 8u : 0u);
}

// Grow the clear box [lo, hi] (sub-blocks; (cm & box) == 0 on entry) along
// x, then y, then z, each as far as it stays clear, towards the sign of
// dir[a] (no growth along an axis with dir 0).  The same box as growing one
// sub-block at a time.
template <class F>
MVF_HD void grow_clear_box(uint64_t cm, int lo[3], int hi[3], const F dir[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (!(dir[a] > F(0)) && !(dir[a] < F(0))) continue;
        int l2[3] = {lo[0], lo[1], lo[2]}, h2[3] = {hi[0], hi[1], hi[2]};
        l2[a] = 0;
        h2[a] = 3;
        const uint64_t m = cm & subblock_box(l2, h2);
        const uint32_t occ = a == 0 ? occupancy_x(m) : a == 1 ? occupancy_y(m) : occupancy_z(m);
        if (dir[a] > F(0)) {
            const uint32_t up = occ & (0xfu << (hi[a] + 1)) & 0xfu;
            hi[a] = up ? __builtin_ctz(up) - 1 : 3;
        } else {
            const uint32_t down = occ & ((1u << lo[a]) - 1u);
            lo[a] = down ? 32 - __builtin_clz(down) : 0;
        }
    }
}

// A mask moved by one sub-block towards -x, -y or -z: sub-block s takes
// sub-block s + 1 of m; the last one takes sub-block 0 of the neighbour
// brick's mask n.
MVF_HD uint64_t sub_shift_x(uint64_t m, uint64_t n)
{
    return ((m >> 1) & 0x7777777777777777ull) | ((n & 0x1111111111111111ull) << 3);
}
MVF_HD uint64_t sub_shift_y(uint64_t m, uint64_t n)
{
    return ((m >> 4) & 0x0fff0fff0fff0fffull) | ((n & 0x000f000f000f000full) << 12);
}
MVF_HD uint64_t sub_shift_z(uint64_t m, uint64_t n)
{
    return (m >> 16) | ((n & 0xffffull) << 48);
}

// Cell mask of a brick from the sub-block flags M[dz][dy][dx] of the brick
// (M[0][0][0]) and of its +x, +y, +z neighbours (0 outside the volume): a
// cell sub-block is set if one of the sub-blocks s .. s + 1 per axis is.
MVF_HD uint64_t cell_mask(const uint64_t M[2][2][2])
{
    uint64_t Ax[2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy) Ax[dz][dy] = M[dz][dy][0] | sub_shift_x(M[dz][dy][0], M[dz][dy][1]);
    uint64_t Ay[2];
    for (int dz = 0; dz < 2; ++dz) Ay[dz] = Ax[dz][0] | sub_shift_y(Ax[dz][0], Ax[dz][1]);
    return Ay[0] | sub_shift_z(Ay[0], Ay[1]);
}

}  // namespace mvf
