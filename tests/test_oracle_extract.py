"""Pins for the oracle's surface points (Input and Output: vertices V and
normals N, at most one vertex per voxel; Metrics: a voxel the surface
crosses gets a vertex).  Each case fixes the answer from geometry, not from
the oracle's own formula."""
import numpy as np
import pytest

import oracle as O

S = 1.0 / 64.0


def _vol(dims, F, W=None, off=(0, 0, 0)):
    nx, ny, nz = dims
    v = O.OVolume.empty(dims, off)
    v.F[...] = F
    v.W[...] = 1 if W is None else W
    return v


def _centres(dims, off, grid):
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    o = np.asarray(grid.arr4()[:3], np.float64)
    s = float(np.float32(grid.voxel_size))
    return (o[0] + s * (x + off[0] + 0.5), o[1] + s * (y + off[1] + 0.5), o[2] + s * (z + off[2] + 0.5))


def test_axis_plane_one_layer_exact():
    """F = (z - z0) / mu with z0 between two voxel layers: exactly the
    voxels of the lower layer whose cell lies in the volume get a vertex,
    on the plane, with normal +z."""
    dims = (12, 10, 9)
    grid = O.OGrid((0.0, 0.0, 0.0), S, 4.0)
    cx, cy, cz = _centres(dims, (0, 0, 0), grid)
    z0 = S * 4.25  # between the centres of layers 3 (3.5 s) and 4 (4.5 s)
    mu = 4 * S
    r = O.extract(_vol(dims, (cz - z0) / mu), grid)
    assert r["n"] == (12 - 1) * (10 - 1)
    assert np.all(r["G"][:, 2] == 3)
    assert np.abs(r["V"][:, 2] - z0).max() < 1e-6 * S
    np.testing.assert_allclose(r["N"], np.tile([0.0, 0.0, 1.0], (r["n"], 1)), atol=1e-12)
    # the voxel's own x and y; global voxel order z, y, x
    gy, gx = np.meshgrid(np.arange(9), np.arange(11), indexing="ij")
    np.testing.assert_array_equal(r["G"][:, 0], gx.reshape(-1))
    np.testing.assert_array_equal(r["G"][:, 1], gy.reshape(-1))
    np.testing.assert_allclose(r["V"][:, 0], S * (r["G"][:, 0] + 0.5), atol=1e-15)


def test_tilted_plane_first_changing_edge():
    """A tilted plane (no voxel centre within 1e-3 voxel of it): the
    vertices are exactly the voxels with a sign change on a +x, +y or +z
    edge (brute force in binary64), each on the first such edge in the
    order x, y, z, lying on the plane with the plane's normal."""
    dims = (16, 15, 14)
    off = (3, -2, 5)
    grid = O.OGrid((-0.1, 0.05, -0.2), S, 4.0)
    n = np.array([0.36, -0.48, 0.8])  # unit
    cx, cy, cz = _centres(dims, off, grid)
    P = np.stack([cx, cy, cz], -1)
    d = float(P[7, 7, 8] @ n) + 0.3141 * S
    phi = (P @ n - d) / (16 * S)
    assert np.abs(phi * 16).min() > 1e-3 and np.abs(phi).max() < 1  # no centre on the plane; all in the band
    r = O.extract(_vol(dims, phi, off=off), grid)
    # brute force: sign changes on the three edges leaving each voxel
    pos = phi > 0
    expect = []
    for z in range(dims[2] - 1):
        for y in range(dims[1] - 1):
            for x in range(dims[0] - 1):
                for a, (dx, dy, dz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    if pos[z, y, x] != pos[z + dz, y + dy, x + dx]:
                        expect.append((x + off[0], y + off[1], z + off[2], a))
                        break
    assert r["n"] == len(expect) > 100
    np.testing.assert_array_equal(r["G"], np.array([e[:3] for e in expect]))
    # the vertex lies on its edge and on the plane
    rel = (r["V"] - np.asarray(grid.arr4()[:3], np.float64)) / float(np.float32(S)) - r["G"] - 0.5
    for i, e in enumerate(expect):
        a = e[3]
        assert 0.0 <= rel[i, a] < 1.0
        assert np.all(np.abs(np.delete(rel[i], a)) < 1e-9)
    assert np.abs(r["V"] @ n - d).max() < 1e-6 * S
    np.testing.assert_allclose(r["N"], np.tile(n, (r["n"], 1)), atol=1e-6)


def test_sphere_points_on_sphere():
    """A sphere's distance field (truncated at 4 voxels): every vertex lies
    within s^2 / (4 R) + rounding of the sphere (linear interpolation of a
    distance along a chord); the normal, a gradient taken over one cell,
    within the turn of the radial direction across a cell (sqrt(3) s / R
    rad) everywhere and within s / R rad at the median; at most one vertex per voxel
    and none beyond the cells the sphere crosses."""
    dims = (40, 40, 40)
    grid = O.OGrid((0.0, 0.0, 0.0), S, 4.0)
    cx, cy, cz = _centres(dims, (0, 0, 0), grid)
    c0 = np.array([20.3, 19.6, 20.1]) * S
    R = 13.7 * S
    dist = np.sqrt((cx - c0[0]) ** 2 + (cy - c0[1]) ** 2 + (cz - c0[2]) ** 2) - R
    F = np.clip(dist / (4 * S), -1, 1)
    r = O.extract(_vol(dims, F), grid)
    assert len({tuple(g) for g in r["G"]}) == r["n"] > 1000
    err = np.abs(np.linalg.norm(r["V"] - c0, axis=1) - R)
    assert err.max() <= S * S / (4 * R) + 1e-6 * S
    radial = (r["V"] - c0) / np.linalg.norm(r["V"] - c0, axis=1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip(np.sum(radial * r["N"], 1), -1, 1)))
    assert ang.max() < np.degrees(np.sqrt(3) * S / R)
    assert np.median(ang) < np.degrees(S / R)
    # every emitting voxel's cell straddles the sphere
    g = r["G"]
    lo = np.linalg.norm(S * (g + 0.5) - c0, axis=1) - R
    assert np.all(np.abs(lo) <= np.sqrt(3) * S + 1e-12)


def test_unobserved_corner_and_truncated_ends():
    """A voxel with W = 0 removes the vertices of the (up to 8) cells that
    have it as a corner, and nothing else; an edge with a truncated end
    (F = 1) gives no vertex."""
    dims = (10, 10, 10)
    grid = O.OGrid((0.0, 0.0, 0.0), S, 4.0)
    cx, cy, cz = _centres(dims, (0, 0, 0), grid)
    F = (cz - 5.25 * S) / (4 * S)  # the layer z = 4 emits
    full = O.extract(_vol(dims, F), grid)
    W = np.ones((10, 10, 10), np.uint16)
    W[4, 6, 3] = 0  # voxel (x 3, y 6, z 4)
    holed = O.extract(_vol(dims, F, W), grid)
    gone = {tuple(g) for g in full["G"]} - {tuple(g) for g in holed["G"]}
    assert gone == {(x, y, 4) for x in (2, 3) for y in (5, 6)}  # cells at z 3 emit nothing anyway
    F2 = F.copy()
    F2[5, 2, 2] = 1.0  # the upper end of voxel (2, 2, 4)'s z edge is truncated
    trunc = O.extract(_vol(dims, F2), grid)
    assert {tuple(g) for g in full["G"]} - {tuple(g) for g in trunc["G"]} == {(2, 2, 4)}


def test_tiles_give_the_single_volumes_points():
    """Two tiles sharing two voxel layers: their points, merged by global
    voxel, are the single volume's points, bit for bit (a voxel of the
    shared layer emits in both tiles with the same value)."""
    dims = (20, 12, 11)
    grid = O.OGrid((0.0, 0.0, 0.0), S, 4.0)
    cx, cy, cz = _centres(dims, (0, 0, 0), grid)
    c0 = np.array([9.7, 6.2, 5.1]) * S
    F = np.clip((np.sqrt((cx - c0[0]) ** 2 + (cy - c0[1]) ** 2 + (cz - c0[2]) ** 2) - 4.4 * S) / (4 * S), -1, 1)
    one = O.extract(_vol(dims, F), grid)
    a = O.extract(_vol((11, 12, 11), F[:, :, :11]), grid)
    b = O.extract(_vol((11, 12, 11), F[:, :, 9:], off=(9, 0, 0)), grid)
    merged = {}
    for r in (a, b):
        for g, v, nn in zip(map(tuple, r["G"]), r["V"], r["N"]):
            if g in merged:
                assert np.array_equal(merged[g][0], v) and np.array_equal(merged[g][1], nn)
            merged[g] = (v, nn)
    assert set(merged) == {tuple(g) for g in one["G"]}
    for g, v, nn in zip(map(tuple, one["G"]), one["V"], one["N"]):
        assert np.array_equal(merged[g][0], v) and np.array_equal(merged[g][1], nn)
