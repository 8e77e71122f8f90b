"""Sub-block masks used for exact empty-space skipping in the raycast:
bit operations checked against brute-force definitions, and soundness of
the cell mask (every cell with a flagged corner voxel is covered)."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_07106_amd", "csrc")


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp(prefix="mvf_masks_")
    so = os.path.join(d, "libmaskshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "native", "mask_shim.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    L.t_subblock_bits.argtypes = [C.c_uint64]
    L.t_subblock_bits.restype = C.c_uint32
    L.t_subblock_box.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.t_subblock_box.restype = C.c_uint64
    L.t_cell_mask.argtypes = [C.POINTER(C.c_uint64)]
    L.t_cell_mask.restype = C.c_uint64
    L.t_grow_clear_box.argtypes = [C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_float)]
    L.t_grow_clear_box.restype = None
    return L


def bit(s):
    x, y, z = s
    return 1 << (z * 16 + y * 4 + x)


def test_subblock_bits(lib):
    rng = np.random.default_rng(1)
    for _ in range(2000):
        b = int(rng.integers(0, 2**63)) | (int(rng.integers(0, 2)) << 63)
        b &= int(rng.integers(0, 2**63))  # sparser patterns too
        want = 0
        for y2 in range(4):
            for x2 in range(4):
                if any((b >> (8 * (2 * y2 + dy) + 2 * x2 + dx)) & 1 for dy in (0, 1) for dx in (0, 1)):
                    want |= 1 << (4 * y2 + x2)
        assert lib.t_subblock_bits(b) == want


def test_subblock_box(lib):
    for lo0 in range(4):
        for hi0 in range(lo0, 4):
            for lo1 in range(4):
                for hi1 in range(lo1, 4):
                    for lo2 in range(4):
                        for hi2 in range(lo2, 4):
                            lo = (C.c_int * 3)(lo0, lo1, lo2)
                            hi = (C.c_int * 3)(hi0, hi1, hi2)
                            want = 0
                            for z in range(lo2, hi2 + 1):
                                for y in range(lo1, hi1 + 1):
                                    for x in range(lo0, hi0 + 1):
                                        want |= bit((x, y, z))
                            assert lib.t_subblock_box(lo, hi) == want


def _fmask_from_flags(lib, fl):
    """The integration's reduction: per pair of z-slices, one bit per voxel
    column (8 y + x), folded by subblock_bits.  fl: bool [8, 8, 8] as [z, y, x]."""
    m = 0
    for zp in range(4):
        cols = fl[2 * zp] | fl[2 * zp + 1]
        b = 0
        for y in range(8):
            for x in range(8):
                if cols[y, x]:
                    b |= 1 << (8 * y + x)
        m |= lib.t_subblock_bits(b) << (16 * zp)
    return m


def test_fmask_and_cell_mask_cover_flagged_corners(lib):
    rng = np.random.default_rng(2)
    nb = 3
    n = 8 * nb
    for trial in range(6):
        fl = rng.random((n, n, n)) < (0.002 if trial % 2 else 0.02)   # [z, y, x]
        fm = np.zeros((nb, nb, nb), np.uint64)   # [bx, by, bz]
        for bx in range(nb):
            for by in range(nb):
                for bz in range(nb):
                    blk = fl[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
                    m = _fmask_from_flags(lib, blk)
                    # brute force: sub-block flag = any voxel of the 2^3 sub-block
                    want = 0
                    for z2 in range(4):
                        for y2 in range(4):
                            for x2 in range(4):
                                if blk[2 * z2:2 * z2 + 2, 2 * y2:2 * y2 + 2, 2 * x2:2 * x2 + 2].any():
                                    want |= bit((x2, y2, z2))
                    assert m == want
                    fm[bx, by, bz] = m
        cm = np.zeros_like(fm)
        for bx in range(nb):
            for by in range(nb):
                for bz in range(nb):
                    m8 = (C.c_uint64 * 8)()
                    for i in range(8):
                        dz, dy, dx = i >> 2, (i >> 1) & 1, i & 1
                        x, y, z = bx + dx, by + dy, bz + dz
                        m8[i] = int(fm[x, y, z]) if (x < nb and y < nb and z < nb) else 0
                    cm[bx, by, bz] = lib.t_cell_mask(m8)
        # every cell (base i, corners i..i+1) with a flagged corner is covered
        # by the cell-mask bit of its base sub-block; and the mask is exactly
        # the one-sub-block dilation of the flags
        sub = np.zeros((4 * nb + 1,) * 3, bool)  # global sub-block flags [x, y, z]
        for X in range(4 * nb):
            for Y in range(4 * nb):
                for Z in range(4 * nb):
                    sub[X, Y, Z] = fl[2 * Z:2 * Z + 2, 2 * Y:2 * Y + 2, 2 * X:2 * X + 2].any()
        for X in range(4 * nb):
            for Y in range(4 * nb):
                for Z in range(4 * nb):
                    got = (int(cm[X // 4, Y // 4, Z // 4]) >> ((Z % 4) * 16 + (Y % 4) * 4 + X % 4)) & 1
                    assert got == int(sub[X:X + 2, Y:Y + 2, Z:Z + 2].any())
        for x in range(n - 1):
            for y in range(n - 1):
                for z in range(n - 1):
                    if fl[z:z + 2, y:y + 2, x:x + 2].any():
                        X, Y, Z = x // 2, y // 2, z // 2
                        assert (int(cm[X // 4, Y // 4, Z // 4]) >> ((Z % 4) * 16 + (Y % 4) * 4 + X % 4)) & 1


def _box_bits(lo, hi):
    m = 0
    for z in range(lo[2], hi[2] + 1):
        for y in range(lo[1], hi[1] + 1):
            for x in range(lo[0], hi[0] + 1):
                m |= bit((x, y, z))
    return m


def test_grow_clear_box_matches_stepwise_growth(lib):
    """The raycast's skip box: from a clear sub-block, grown along x, then y,
    then z towards the ray direction one sub-block at a time while it stays
    clear (brute force here) -- the helper reaches the same box directly."""
    rng = np.random.default_rng(5)
    n = 0
    for trial in range(3000):
        dens = (0.02, 0.1, 0.3)[trial % 3]
        cm = 0
        for b in range(64):
            if rng.random() < dens:
                cm |= 1 << b
        s = [int(v) for v in rng.integers(0, 4, 3)]
        if cm & bit(s):
            continue
        d = [float(rng.choice([-1.0, 0.0, 1.0])) for _ in range(3)]
        lo, hi = list(s), list(s)
        for a in range(3):
            if d[a] > 0:
                while hi[a] < 3:
                    hi[a] += 1
                    if cm & _box_bits(lo, hi):
                        hi[a] -= 1
                        break
            elif d[a] < 0:
                while lo[a] > 0:
                    lo[a] -= 1
                    if cm & _box_bits(lo, hi):
                        lo[a] += 1
                        break
        clo, chi = (C.c_int * 3)(*s), (C.c_int * 3)(*s)
        lib.t_grow_clear_box(cm, clo, chi, (C.c_float * 3)(*d))
        assert (list(clo), list(chi)) == (lo, hi), (hex(cm), s, d)
        assert cm & _box_bits(lo, hi) == 0
        n += 1
    assert n > 1000
