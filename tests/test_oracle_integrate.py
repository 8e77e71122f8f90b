"""Pins for the oracle's volumetric integration (Volumetric Integration
section of the paper, Algorithm 1's per-voxel loop).

Each test checks the oracle against something other than its own formula:
closed forms on exactly representable geometry, the geometry of a plane,
the paper's tiled-equals-single invariant (Comparison to KinectFusion), and
algebraic identities of a running average."""
import math

import numpy as np
import pytest

import oracle as O
from synth import scenes as S

S64 = 1.0 / 64.0  # exact binary voxel size


def _axis_setup(depth_value, w=32, h=24, gx0=40, gy0=-20, tz=-0.2578125, nz=64, z0=0):
    """Camera looking down world +z (R = I) whose optical axis passes through
    the centres of voxel column (gx0, gy0); principal point on a pixel centre.
    Everything is exactly representable, so the on-axis projective distance
    is exact: the voxel is on the pixel ray through (cx, cy), whose length
    factor is exactly 1."""
    grid = O.OGrid((0.0, 0.0, 0.0), S64, 4.0, 128)
    T = np.zeros((3, 4))
    T[:, :3] = np.eye(3)
    T[:, 3] = [S64 * (gx0 + 0.5), S64 * (gy0 + 0.5), tz]
    K = np.array([100.0, 100.0, 16.0, 12.0], np.float32)
    vol = O.OVolume.empty((8, 8, nz), (gx0 - 4, gy0 - 4, z0))
    depth = np.full((h, w), depth_value, np.float32)
    return grid, T, K, vol, depth


def _axis_expected(Z0, tz, nz, z0, mu):
    gz = z0 + np.arange(nz)
    pz = S64 * (gz + 0.5) - tz
    sdf = Z0 - pz
    upd = sdf >= -mu
    F = np.where(upd, np.minimum(1.0, sdf / mu), 0.0)
    return F, upd.astype(np.uint16), sdf


def test_on_axis_closed_form():
    """F = min(1, (D - z)/mu) and W = 1 on the optical axis; no update more
    than mu behind the surface; the boundary voxel sdf = -mu is updated."""
    Z0, tz = 0.5, -0.2578125
    grid, T, K, vol, depth = _axis_setup(Z0, tz=tz)
    O.integrate(vol, grid, depth, None, K, T)
    F_exp, W_exp, sdf = _axis_expected(Z0, tz, 64, 0, grid.mu)
    assert grid.mu == 4 * S64
    # the truncation boundary is hit exactly by one voxel
    assert np.any(sdf == -grid.mu)
    col_F = vol.F[:, 4, 4]
    col_W = vol.W[:, 4, 4]
    np.testing.assert_array_equal(col_W, W_exp)
    np.testing.assert_array_equal(col_F, F_exp)
    # free space in front of the surface is clamped to exactly +1
    assert np.sum(col_F == 1.0) > 10 and np.sum(col_W == 0) > 10


def test_on_axis_with_z_offset_volume():
    """The same column stored in a volume whose translation h_t is non-zero
    along z gives the same values for the same global voxels."""
    Z0, tz = 0.5, -0.2578125
    grid, T, K, vol, depth = _axis_setup(Z0, tz=tz, nz=24, z0=20)
    O.integrate(vol, grid, depth, None, K, T)
    F_exp, W_exp, _ = _axis_expected(Z0, tz, 24, 20, grid.mu)
    np.testing.assert_array_equal(vol.W[:, 4, 4], W_exp)
    np.testing.assert_array_equal(vol.F[:, 4, 4], F_exp)


def test_fuse_twice_exact():
    """Fusing the same frame twice from empty leaves F unchanged bit for bit
    and doubles the integer weights (spec invariant)."""
    seq = S.small_room_sequence(noise=True)
    grid = O.OGrid((-1.0, -1.0, -1.0), 2.0 / 48, 4.0, 128)
    vol = O.OVolume.empty((48, 48, 48))
    d, rgb = seq.frame(3)
    O.integrate(vol, grid, d, rgb, seq.K.as_array(), seq.poses[3])
    F1, W1, C1 = vol.F.copy(), vol.W.copy(), vol.Cc.copy()
    assert W1.max() == 1 and (W1 > 0).sum() > 1000
    O.integrate(vol, grid, d, rgb, seq.K.as_array(), seq.poses[3])
    np.testing.assert_array_equal(vol.W, 2 * W1)
    np.testing.assert_array_equal(vol.F, F1)
    np.testing.assert_array_equal(vol.Cc[..., :3], C1[..., :3])
    np.testing.assert_array_equal(vol.Cc[..., 3], 2 * C1[..., 3])


def test_running_mean_of_frames():
    """Frames of fronto-parallel planes at different depths: the fused value
    of an on-axis voxel is the mean of the per-frame truncated distances."""
    tz = -0.2578125
    depths = [0.5, 0.53125, 0.46875, 0.5625, 0.515625]
    grid, T, K, vol, _ = _axis_setup(depths[0], tz=tz)
    phis = []
    for Z0 in depths:
        O.integrate(vol, grid, np.full((24, 32), Z0, np.float32), None, K, T)
        phis.append(_axis_expected(Z0, tz, 64, 0, grid.mu))
    all_upd = np.all([p[1] == 1 for p in phis], axis=0)
    assert all_upd.sum() > 10
    mean = np.mean([p[0] for p in phis], axis=0)
    col = vol.F[:, 4, 4]
    np.testing.assert_allclose(col[all_upd], mean[all_upd], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(vol.W[:, 4, 4][all_upd], len(depths))


def test_weight_saturation():
    """The running weight stops at w_max; identical frames keep F fixed."""
    grid, T, K, vol, depth = _axis_setup(0.5)
    grid.w_max = 3
    for _ in range(6):
        O.integrate(vol, grid, depth, None, K, T)
    F_exp, W_exp, _ = _axis_expected(0.5, -0.2578125, 64, 0, grid.mu)
    np.testing.assert_array_equal(vol.W[:, 4, 4], 3 * W_exp)
    np.testing.assert_allclose(vol.F[:, 4, 4], F_exp, atol=1e-15)


@pytest.mark.parametrize("bad", [0.0, -1.0, np.nan, np.inf, -np.inf])
def test_invalid_depth_no_update(bad):
    grid, T, K, vol, depth = _axis_setup(0.5)
    depth[:] = bad
    st = O.integrate(vol, grid, depth, None, K, T)
    assert st == (0, 0, 0)
    assert vol.W.max() == 0 and np.all(vol.F == 0)


def test_behind_camera_and_outside_image_no_update():
    grid, T, K, vol, depth = _axis_setup(0.5)
    # camera beyond the whole volume looking further along +z: p_z < 0
    T2 = T.copy()
    T2[2, 3] = 5.0
    assert O.integrate(vol, grid, depth, None, K, T2) == (0, 0, 0)
    # volume far off to the side: every voxel projects outside the image
    vol2 = O.OVolume.empty((8, 8, 8), (400, 0, 40))
    assert O.integrate(vol2, grid, depth, None, K, T) == (0, 0, 0)
    assert vol.W.max() == 0 and vol2.W.max() == 0


def test_colour_band_and_rounded_mean():
    """Colour is fused only within |dist| <= mu (the band boundary dist = mu
    is included), as a rounded running mean with its own weight."""
    Z0, tz = 0.5, -0.2578125
    grid, T, K, vol, depth = _axis_setup(Z0, tz=tz)
    rgb1 = np.zeros((24, 32, 3), np.uint8)
    rgb1[:] = (10, 200, 77)
    rgb2 = np.zeros_like(rgb1)
    rgb2[:] = (30, 100, 255)
    O.integrate(vol, grid, depth, rgb1, K, T)
    _, _, sdf = _axis_expected(Z0, tz, 64, 0, grid.mu)
    band = np.abs(sdf) <= grid.mu
    assert np.any(sdf == grid.mu) and np.any(sdf == -grid.mu)
    col = vol.Cc[:, 4, 4]
    np.testing.assert_array_equal(col[band], np.tile([10, 200, 77, 1], (band.sum(), 1)))
    np.testing.assert_array_equal(col[~band], 0)
    O.integrate(vol, grid, depth, rgb2, K, T)
    col = vol.Cc[:, 4, 4]
    # mean of 10 and 30 is 20; 200,100 -> 150; 77,255 -> 166
    np.testing.assert_array_equal(col[band], np.tile([20, 150, 166, 2], (band.sum(), 1)))


def _plane_depth(K, w, h, n_c, d):
    """z-depth of the plane {x : n_c . x = d} (camera frame) at every pixel."""
    u, v = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    r = np.stack([(u - K[2]) / K[0], (v - K[3]) / K[1], np.ones_like(u)], -1)
    t = d / (r @ n_c)
    return np.where(t > 0, t, 0.0).astype(np.float32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_projective_distance_matches_plane_geometry(seed):
    """One noise-free frame of a tilted plane seen from a rotated camera: for
    every voxel whose value is not clamped, mu F equals the true signed
    distance to the plane divided by the cosine of the angle between the
    voxel's view ray and the plane normal, up to the pixel quantisation
    term d eps / (c_r c_p) with eps = 0.75 / f.  A z-depth-for-range mix-up,
    a dropped ray-length factor, a transposed rotation or a sign error all
    break this bound by orders of magnitude."""
    rng = np.random.default_rng(seed)
    w, h = 160, 120
    K = np.array([150.0, 150.0, 79.5, 59.5], np.float32)
    f = 150.0
    s = 0.02
    grid = O.OGrid((-0.9, -0.7, -0.8), s, 4.0, 128)
    mu = grid.mu
    eye = rng.uniform(-0.2, 0.2, 3) + np.array([0.0, 0.0, -1.2])
    T = S.look_at(eye, rng.uniform(-0.1, 0.1, 3), up=(0, -1, 0.2))
    R, C = T[:, :3], T[:, 3]
    # plane through a point near the volume centre, normal facing the camera
    n_w = rng.normal(size=3) * 0.3 + (C - 0.0)
    n_w /= np.linalg.norm(n_w)
    x0 = rng.uniform(-0.1, 0.1, 3)
    n_c = R.T @ n_w
    d = float(n_w @ (x0 - C))  # < 0: camera on the +n side
    # write the plane as n'.x = d' with d' > 0 in the camera frame
    n_c, d = -n_c, -d
    assert d > 0
    depth = _plane_depth(K, w, h, n_c, d)
    off = (3, 5, 2)
    vol = O.OVolume.empty((64, 60, 70), off)
    O.integrate(vol, grid, depth, None, K, T)
    nz, ny, nx = vol.W.shape
    gz, gy, gx = np.meshgrid(np.arange(nz) + off[2], np.arange(ny) + off[1],
                             np.arange(nx) + off[0], indexing="ij")
    xw = np.stack([grid.origin[0] + s * (gx + 0.5), grid.origin[1] + s * (gy + 0.5),
                   grid.origin[2] + s * (gz + 0.5)], -1)
    p = (xw - C) @ R  # camera frame
    rho = np.linalg.norm(p, axis=-1)
    c_p = (p @ n_c) / rho
    sdf_true = d - p @ n_c
    sel = (vol.W == 1) & (np.abs(vol.F) < 0.999) & (c_p > 0.3)
    assert sel.sum() > 2000
    eps = 0.75 / f
    bound = d * eps / ((c_p - eps) * c_p) + 2e-5
    err = np.abs(mu * vol.F - sdf_true / c_p)
    assert np.all(err[sel] <= bound[sel]), float((err - bound)[sel].max())
    # and every voxel clearly in front of the plane (within the view) is
    # clamped to +1, every voxel clearly behind beyond mu is untouched
    front = (vol.W == 1) & (sdf_true / c_p > mu + bound)
    assert np.all(vol.F[front] == 1.0)
    behind = (sdf_true / np.maximum(c_p, 1e-9) < -mu - bound) & (c_p > 0.3)
    assert np.all(vol.W[behind] == 0)


def test_tiled_equals_single_volume():
    """The paper's invariant (Comparison to KinectFusion): subvolumes that
    overlap by two voxels, placed on the same global grid, hold exactly the
    voxels the single volume holds."""
    seq = S.small_room_sequence(noise=True)
    n = 32
    grid = O.OGrid((-1.0, -1.0, -1.0), 2.0 / n, 4.0, 128)
    big = O.OVolume.empty((n, n, n))
    half = n // 2
    tiles = [O.OVolume.empty((half + 1,) * 3, (ox, oy, oz))
             for oz in (0, half - 1) for oy in (0, half - 1) for ox in (0, half - 1)]
    for i in (0, 4, 7):
        d, rgb = seq.frame(i)
        O.integrate(big, grid, d, rgb, seq.K.as_array(), seq.poses[i])
        for t in tiles:
            O.integrate(t, grid, d, rgb, seq.K.as_array(), seq.poses[i])
    assert (big.W > 0).mean() > 0.3
    for t in tiles:
        ox, oy, oz = t.offset
        sl = np.s_[oz:oz + half + 1, oy:oy + half + 1, ox:ox + half + 1]
        np.testing.assert_array_equal(t.W, big.W[sl])
        np.testing.assert_array_equal(t.F, big.F[sl])
        np.testing.assert_array_equal(t.Cc, big.Cc[sl])
