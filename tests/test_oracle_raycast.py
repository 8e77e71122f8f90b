"""Pins for the oracle's raycast (Raycasting section of the paper and
Algorithm 1's per-pixel loop; the shared-map nearest-distance rule; the
tiled-equals-single argument of Comparison to KinectFusion).

A volume filled with a linear field makes trilinear interpolation and the
linear refinement between two samples exact, so the raycast depth, vertex
and normal must equal the analytic ray-plane intersection."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S


def _lattice_points(grid, vol):
    nx, ny, nz = vol.dims
    ox, oy, oz = vol.offset
    gz, gy, gx = np.meshgrid(np.arange(nz) + oz, np.arange(ny) + oy, np.arange(nx) + ox,
                             indexing="ij")
    s = grid.voxel_size
    return np.stack([grid.origin[0] + s * (gx + 0.5), grid.origin[1] + s * (gy + 0.5),
                     grid.origin[2] + s * (gz + 0.5)], -1)


def _fill(vol, grid, fn, W=1):
    x = _lattice_points(grid, vol)
    vol.F[:] = fn(x)
    vol.W[:] = W


def _rays_world(K, w, h, T):
    u, v = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    dc = np.stack([(u - K[2]) / K[0], (v - K[3]) / K[1], np.ones_like(u)], -1)
    dh = dc / np.linalg.norm(dc, axis=-1, keepdims=True)
    return dh, dh @ T[:, :3].T


def _inside_box(x, lo, hi, margin):
    return np.all((x > lo + margin) & (x < hi - margin), axis=-1)


def _domain_box(grid, vol):
    s = grid.voxel_size
    o = np.asarray(grid.origin)
    lo = o + s * (np.asarray(vol.offset) + 0.5)
    hi = o + s * (np.asarray(vol.offset) + np.asarray(vol.dims) - 0.5)
    return lo, hi


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_linear_field_exact(seed):
    rng = np.random.default_rng(seed)
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    vol = O.OVolume.empty((64, 64, 64), (0, 0, 0))
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    d0 = float(rng.uniform(-0.2, 0.2))
    mu = grid.mu
    _fill(vol, grid, lambda x: (x @ n - d0) / mu)
    # camera on the positive side, looking at the plane
    C = n * (d0 + rng.uniform(0.8, 1.2)) + rng.uniform(-0.2, 0.2, 3)
    T = S.look_at(C, C - n + rng.uniform(-0.3, 0.3, 3), up=rng.normal(size=3))
    K = np.array([120.0, 120.0, 63.5, 47.5], np.float32)
    w, h = 128, 96
    rc = O.raycast([vol], grid, K, T, w, h)
    dh, dw = _rays_world(K, w, h, T)
    den = dw @ n
    t_hit = np.where(den < 0, (d0 - C @ n) / np.where(den < 0, den, -1.0), np.inf)
    x_hit = C + t_hit[..., None] * dw
    lo, hi = _domain_box(grid, vol)
    must = np.isfinite(t_hit) & _inside_box(x_hit, lo, hi, 1.5 * grid.voxel_size)
    never = ~np.isfinite(t_hit) | ~_inside_box(x_hit, lo, hi, -1.5 * grid.voxel_size)
    hit = rc["hit"] >= 0
    assert must.sum() > 3000
    assert np.all(hit[must]) and not np.any(hit[never])
    np.testing.assert_allclose(rc["depth"][must], (t_hit * dh[..., 2])[must], atol=1e-5, rtol=0)
    np.testing.assert_allclose(rc["vertex"][must], x_hit[must], atol=1e-5, rtol=0)
    np.testing.assert_allclose(rc["normal"][must], np.broadcast_to(n, x_hit.shape)[must],
                               atol=1e-5, rtol=0)
    assert np.all(rc["depth"][~hit] == 0) and np.all(np.isnan(rc["normal"][~hit]))


def test_sphere_field_close_to_analytic():
    """A truncated distance field of a sphere: the zero crossing found by the
    march lies within a small fraction of a voxel of the analytic surface."""
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    vol = O.OVolume.empty((64, 64, 64))
    c = np.array([0.05, -0.1, 0.1])
    r = 0.45
    mu = grid.mu
    _fill(vol, grid, lambda x: np.clip((np.linalg.norm(x - c, axis=-1) - r) / mu, -1, 1))
    T = S.look_at([0.2, -0.9, 0.3], c, up=(0, 0, 1))
    K = np.array([120.0, 120.0, 63.5, 47.5], np.float32)
    w, h = 128, 96
    rc = O.raycast([vol], grid, K, T, w, h)
    dh, dw = _rays_world(K, w, h, T)
    C = T[:, 3]
    oc = C - c
    b = dw @ oc
    disc = b * b - (oc @ oc - r * r)
    t_hit = np.where(disc > 0, -b - np.sqrt(np.maximum(disc, 0)), np.inf)
    x_hit = C + t_hit[..., None] * dw
    nrm = (x_hit - c) / r
    cosang = -np.einsum("ijk,ijk->ij", nrm, dw)
    good = np.isfinite(t_hit) & (cosang > 0.3)
    assert good.sum() > 2000
    hit = rc["hit"] >= 0
    assert np.all(hit[good])
    err = np.abs(rc["depth"] - t_hit * dh[..., 2])[good]
    assert err.max() < 0.15 * grid.voxel_size, err.max() / grid.voxel_size
    # the gradient of a trilinear patch of a sampled distance field deviates
    # from the analytic normal by O(s / r); worst case a few degrees
    ang = np.einsum("ijk,ijk->ij", rc["normal"], nrm)[good]
    assert ang.min() > np.cos(np.deg2rad(5.0))
    assert np.median(ang) > np.cos(np.deg2rad(2.0))
    # rays that miss the sphere by more than two voxels find nothing
    miss = (disc < 0) & (np.abs(np.sqrt(np.maximum(oc @ oc - b * b, 0)) - r) > 2 * grid.voxel_size)
    assert not np.any(hit[miss])


def test_first_front_face_only():
    """A slab of negative values between two parallel planes: the ray stops
    at the near face; the far face (a minus-to-plus change) never counts, and
    a camera inside the slab sees nothing."""
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    vol = O.OVolume.empty((64, 64, 64))
    mu = grid.mu
    _fill(vol, grid, lambda x: (np.abs(x[..., 2] - 0.0) - 0.2) / mu)
    K = np.array([100.0, 100.0, 31.5, 23.5], np.float32)
    T = S.look_at([0.0, 0.0, 0.8], [0.0, 0.0, 0.0], up=(0, 1, 0))
    rc = O.raycast([vol], grid, K, T, 64, 48)
    hit = rc["hit"] >= 0
    assert hit.all()
    np.testing.assert_allclose(rc["vertex"][..., 2], 0.2, atol=1e-5)
    T_in = S.look_at([0.0, 0.0, 0.1], [0.0, 0.0, -1.0], up=(0, 1, 0))
    rc2 = O.raycast([vol], grid, K, T_in, 64, 48)
    assert not np.any(rc2["hit"] >= 0)


def test_unobserved_voxels_block_crossings():
    """A sample is valid only if all 8 voxels of its cell were observed."""
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    vol = O.OVolume.empty((64, 64, 64))
    mu = grid.mu
    _fill(vol, grid, lambda x: (x[..., 2] - 0.0) / mu)
    x = _lattice_points(grid, vol)
    hole = (np.abs(x[..., 0]) < 0.25) & (np.abs(x[..., 1]) < 0.25)
    vol.W[hole] = 0
    vol.F[hole] = 0.0
    K = np.array([40.0, 40.0, 31.5, 23.5], np.float32)
    T = S.look_at([0.0, 0.0, 0.9], [0.0, 0.0, 0.0], up=(0, 1, 0))
    rc = O.raycast([vol], grid, K, T, 64, 48)
    dh, dw = _rays_world(K, 64, 48, T)
    t = -0.9 / dw[..., 2]
    xh = T[:, 3] + t[..., None] * dw
    in_hole = (np.abs(xh[..., 0]) < 0.25 - 2 / 32) & (np.abs(xh[..., 1]) < 0.25 - 2 / 32)
    outside = (np.abs(xh[..., 0]) > 0.25 + 2 / 32) | (np.abs(xh[..., 1]) > 0.25 + 2 / 32)
    hit = rc["hit"] >= 0
    assert in_hole.sum() > 50 and outside.sum() > 50
    assert not np.any(hit[in_hole]) and np.all(hit[outside])


def test_nearest_surface_wins_across_volumes():
    """All volumes write one shared map; the shortest raycast distance wins
    (Raycasting section), whatever the order of the volumes."""
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    mu = grid.mu
    near = O.OVolume.empty((24, 24, 24), (20, 20, 40))  # |x|,|y| < 0.375, z in [0.25, 1.0]
    far = O.OVolume.empty((64, 64, 24), (0, 0, 0))     # z in [-1, -0.25]
    _fill(near, grid, lambda x: (x[..., 2] - 0.5) / mu)
    _fill(far, grid, lambda x: (x[..., 2] + 0.6) / mu)
    K = np.array([60.0, 60.0, 31.5, 23.5], np.float32)
    T = S.look_at([0.05, -0.03, 1.6], [0.0, 0.0, 0.0], up=(0, 1, 0))
    a = O.raycast([near, far], grid, K, T, 64, 48)
    b = O.raycast([far, near], grid, K, T, 64, 48)
    ha, hb = a["hit"] >= 0, b["hit"] >= 0
    np.testing.assert_array_equal(ha, hb)
    np.testing.assert_array_equal(a["depth"], b["depth"])
    # pixels that see the near plane report it; others the far plane
    za = a["vertex"][..., 2]
    assert np.sum(np.abs(za[ha] - 0.5) < 1e-5) > 500
    assert np.sum(np.abs(za[ha] + 0.6) < 1e-5) > 100
    assert np.all((np.abs(za[ha] - 0.5) < 1e-5) | (np.abs(za[ha] + 0.6) < 1e-5))
    near_px = np.abs(za - 0.5) < 1e-5
    np.testing.assert_array_equal(a["hit"][near_px], 0)
    np.testing.assert_array_equal(b["hit"][near_px], 1)


def test_tiled_equals_single_raycast():
    """Subvolumes overlapping by two voxels reproduce the single volume's
    depth, vertex and normal maps (Comparison to KinectFusion): the binary32
    crossing distance is bit-identical and the binary64 outputs agree to
    rounding."""
    seq = S.small_room_sequence(noise=True)
    n = 32
    grid = O.OGrid((-1.0, -1.0, -1.0), 2.0 / n, 4.0, 128)
    big = O.OVolume.empty((n, n, n))
    half = n // 2
    tiles = [O.OVolume.empty((half + 1,) * 3, (ox, oy, oz))
             for oz in (0, half - 1) for oy in (0, half - 1) for ox in (0, half - 1)]
    K = seq.K.as_array()
    for i in range(10):
        d, rgb = seq.frame(i)
        O.integrate(big, grid, d, rgb, K, seq.poses[i])
        for t in tiles:
            O.integrate(t, grid, d, rgb, K, seq.poses[i])
    for pose in (seq.poses[9], seq.poses[2]):
        a = O.raycast([big], grid, K, pose, 320, 240)
        b = O.raycast(tiles, grid, K, pose, 320, 240)
        ha, hb = a["hit"] >= 0, b["hit"] >= 0
        assert ha.mean() > 0.2
        np.testing.assert_array_equal(ha, hb)
        np.testing.assert_array_equal(a["tstar"], b["tstar"])
        np.testing.assert_allclose(a["depth"], b["depth"], atol=1e-12, rtol=0)
        np.testing.assert_allclose(a["normal"][ha], b["normal"][hb], atol=1e-9, rtol=0)


def test_step_must_be_below_one_voxel():
    grid = O.OGrid((0.0, 0.0, 0.0), 0.1)
    vol = O.OVolume.empty((4, 4, 4))
    with pytest.raises(ValueError):
        O.raycast([vol], grid, np.array([10, 10, 2, 2], np.float32), S.look_at([0, 0, -1], [0, 0, 0]),
                  4, 4, step=1.0)


# -- the normal's cell (the Raycasting section takes the normal as the
# derivative of the TSDF at the zero crossing; the reading: the gradient of
# the trilinear patch of the cell holding the crossing's second sample,
# evaluated at the vertex) -------------------------------------------------

_KINK = dict(a=0.011, b=-0.007, s1=-0.05, s2=-0.4, plane=32, z0=31.7)


def _kink_field(gx, gy, gz):
    """Lattice values piecewise linear along z with a kink at the voxel plane
    gz = plane: slope s1 below it, s2 above, zero of the lower piece at z0
    (on the volume's axis).  Trilinear interpolation of such values is
    linear inside every cell, so a cell's gradient is the closed form
    (a, b, slope of its z interval) in voxel units."""
    k = _KINK
    h = np.where(gz <= k["plane"], k["s1"] * (gz - k["plane"]), k["s2"] * (gz - k["plane"]))
    return k["a"] * (gx - 32) + k["b"] * (gy - 32) + h + (-k["s1"]) * (k["plane"] - k["z0"])


def _kink_setup():
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    vol = O.OVolume.empty((64, 64, 64))
    gz, gy, gx = np.meshgrid(np.arange(64.0), np.arange(64.0), np.arange(64.0), indexing="ij")
    vol.F[:] = _kink_field(gx, gy, gz)
    vol.W[:] = 1
    # camera below the kink looking up through it at a slant, so rays cross
    # the plane at every phase of the sample lattice
    T = S.look_at([0.11, -0.07, -0.55], [-0.05, 0.04, 0.3], up=(0, 1, 0))
    K = np.array([70.0, 70.0, 47.5, 35.5], np.float32)
    return grid, vol, T, K, 96, 72


def _kink_expected(grid, vol, T, K, w, h, step=0.5):
    """Per pixel, from the geometry alone (binary64): the first sample pair
    (k - 1, k) with a plus-to-minus change of the field, the z cells of the
    two samples and of the vertex on the chord between them, and the
    normal of the second sample's cell.  Pixels whose decisive values lie
    within rounding of a cell boundary or of zero are marked unsure."""
    k_ = _KINK
    s = grid.voxel_size
    dh, dw = _rays_world(K, w, h, T)
    C = np.asarray(T)[:, 3]
    delta = step * s
    ks = np.arange(1, int(2.0 / delta))
    x = C[None, None, None, :] + (ks[None, None, :, None] * delta) * dw[:, :, None, :]
    l = (x - np.asarray(grid.origin)) / s - 0.5
    inside = np.all((l >= 0) & (l < 63), axis=-1)
    lz = l[..., 2]
    cz = np.floor(lz)
    slope = np.where(cz < k_["plane"], k_["s1"], k_["s2"])
    # linear inside each cell: value at the cell base plus slope * fraction
    base = np.where(cz < k_["plane"], k_["s1"] * (cz - k_["plane"]), k_["s2"] * (cz - k_["plane"]))
    Fv = (k_["a"] * (l[..., 0] - 32) + k_["b"] * (l[..., 1] - 32) + base + slope * (lz - cz)
          + (-k_["s1"]) * (k_["plane"] - k_["z0"]))
    pos = inside[..., :-1] & inside[..., 1:] & (Fv[..., :-1] > 0) & (Fv[..., 1:] <= 0)
    anyx = pos.any(-1)
    j = np.argmax(pos, axis=-1)  # pair (j, j + 1) of ks
    take = lambda a, o: np.take_along_axis(a, (j + o)[..., None], -1)[..., 0]
    Fa, Fb = take(Fv, 0), take(Fv, 1)
    za, zb = take(lz, 0), take(lz, 1)
    zv = za + (zb - za) * Fa / (Fa - Fb)
    nrm = np.stack([np.full(zb.shape, k_["a"]), np.full(zb.shape, k_["b"]),
                    np.where(np.floor(zb) < k_["plane"], k_["s1"], k_["s2"])], -1)
    nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
    frac = lambda z: np.abs(z - np.round(z))
    unsure = (frac(za) < 1e-4) | (frac(zb) < 1e-4) | (frac(zv) < 1e-4) | (np.abs(Fa) < 1e-4) | (np.abs(Fb) < 1e-4)
    return dict(hit=anyx, cell_a=np.floor(za), cell_b=np.floor(zb), cell_v=np.floor(zv), normal=nrm,
                unsure=unsure)


def _kink_check(rc, ex):
    """Normal error of each sure hit pixel against the closed form."""
    hit = rc["hit"] >= 0
    sure = ex["hit"] & ~ex["unsure"]
    assert np.array_equal(hit[sure], ex["hit"][sure])
    return np.abs(rc["normal"] - ex["normal"]).max(-1), sure


def test_normal_cell_pinned_by_a_kinked_field():
    """Where the sample pair straddles the kink, the three candidate cells
    (first sample's, second sample's, vertex's own) have gradients that
    differ by a closed-form amount; the oracle's normal must be the second
    sample's, including where the vertex lies outside that cell (the patch
    extended linearly)."""
    grid, vol, T, K, w, h = _kink_setup()
    rc = O.raycast([vol], grid, K, T, w, h)
    ex = _kink_expected(grid, vol, T, K, w, h)
    err, sure = _kink_check(rc, ex)
    straddle = sure & (ex["cell_a"] != ex["cell_b"])
    outside = straddle & (ex["cell_v"] != ex["cell_b"])
    assert straddle.sum() > 300 and outside.sum() > 100, (straddle.sum(), outside.sum())
    # the candidates differ by far more than the tolerance
    n1 = np.array([_KINK["a"], _KINK["b"], _KINK["s1"]]); n1 /= np.linalg.norm(n1)
    n2 = np.array([_KINK["a"], _KINK["b"], _KINK["s2"]]); n2 /= np.linalg.norm(n2)
    assert np.abs(n1 - n2).max() > 0.1
    assert err[sure].max() < 1e-5, err[sure].max()


@pytest.mark.parametrize("variant", [0, 2])
def test_kink_pin_rejects_other_cells(tmp_path, variant):
    """The same pin fails for an oracle built with the first sample's cell
    (0) or the vertex's own cell (2) for the normal."""
    lib = O.build_variant({"ORC_NORMAL_CELL": variant}, str(tmp_path))
    grid, vol, T, K, w, h = _kink_setup()
    rc = O.raycast([vol], grid, K, T, w, h, oracle_lib=lib)
    ex = _kink_expected(grid, vol, T, K, w, h)
    err, sure = _kink_check(rc, ex)
    assert (err[sure] > 0.1).sum() > 100
