"""GPU parity of TSDF integration against the CPU oracle (weights and
colour bit-exact, TSDF within 1e-5 truncation units)."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S
from tests.util import compare_volume, dev, fuse_both, log, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


def test_small_room_128(mvf):
    """The plain single-volume workload: 128^3 over a 2 m cube, 10 frames of
    320x240 (f = 262.5) from the seeded room."""
    log("integrate 128^3 small room, 10 frames 320x240")
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 128
    og = O.OGrid(origin, s, 4.0, 128)
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        ids, ovs = fuse_both(ctx, gid, og, [((0, 0, 0), (128, 128, 128))], seq, range(10))
        _, W, _, err = compare_volume(ctx, ids[0], ovs[0])
        st = ctx.stats()
        assert st["voxels_updated"] > 1_000_000
        log(f"small room ok: max |dF| {err:.2e}, updated {st['voxels_updated']}")


@pytest.mark.parametrize("seed", range(6))
def test_random_ragged_volumes(mvf, seed):
    """Random poses, ragged volume dims (not multiples of the 8-voxel brick),
    offsets, intrinsics, image sizes, truncation and weight caps; random
    depth maps with invalid pixels (0, NaN, inf, negative); several frames."""
    rng = np.random.default_rng(100 + seed)
    dims = tuple(int(x) for x in rng.integers(3, 41, 3))
    off = tuple(int(x) for x in rng.integers(-20, 20, 3))
    s = float(rng.uniform(0.01, 0.05))
    origin = tuple(float(x) for x in rng.uniform(-0.5, 0.5, 3))
    trunc = float(rng.choice([1.0, 2.5, 4.0]))
    w_max = int(rng.choice([1, 3, 128, 65535]))
    w, h = int(rng.integers(7, 90)), int(rng.integers(5, 70))
    K = np.array([rng.uniform(20, 120), rng.uniform(20, 120), rng.uniform(0, w), rng.uniform(0, h)], np.float32)
    og = O.OGrid(origin, s, trunc, w_max)
    center = np.asarray(origin) + s * (np.asarray(off) + np.asarray(dims) / 2)
    log(f"integrate ragged seed={seed} dims={dims} off={off} img={w}x{h} wmax={w_max}")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, trunc, w_max)
        vid = ctx.volume(gid, off, dims)
        ov = O.OVolume.empty(dims, off)
        for f in range(4):
            eye = center + rng.normal(size=3) * s * max(dims) * 0.8
            T = S.look_at(eye, center + rng.normal(size=3) * s * 3, up=rng.normal(size=3))
            dist = np.linalg.norm(eye - center)
            depth = (dist + rng.normal(size=(h, w)) * s * max(dims) * 0.4).astype(np.float32)
            bad = rng.uniform(size=(h, w))
            depth[bad < 0.05] = 0.0
            depth[(bad >= 0.05) & (bad < 0.08)] = np.nan
            depth[(bad >= 0.08) & (bad < 0.1)] = np.inf
            depth[(bad >= 0.1) & (bad < 0.12)] = -1.0
            rgb = rng.integers(0, 256, (h, w, 3)).astype(np.uint8)
            use_rgb = f % 2 == 0
            O.integrate(ov, og, depth, rgb if use_rgb else None, K, T)
            ctx.integrate(t(depth), t(rgb) if use_rgb else None, T, K)
        compare_volume(ctx, vid, ov)


def test_empty_and_invalid_frames(mvf):
    """A frame with no valid depth, and a volume outside the view, leave
    every voxel unobserved."""
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 32
    log("integrate empty frame / out-of-view volume")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s)
        a = ctx.volume(gid, (0, 0, 0), (32, 32, 32))
        b = ctx.volume(gid, (400, 400, 400), (16, 16, 16))
        d = np.zeros((240, 320), np.float32)
        ctx.integrate(t(d), None, seq.poses[0], seq.K.as_array())
        d2, _ = seq.frame(0)
        ctx.integrate(t(d2), None, seq.poses[0], seq.K.as_array())
        _, Wa, _ = ctx.read_volume(a)
        _, Wb, _ = ctx.read_volume(b)
        assert Wa.max() == 1 and Wb.max() == 0


def test_fuse_twice_exact_on_gpu(mvf):
    """Fusing the same frame twice from empty leaves F unchanged bit for bit
    and doubles W (on the device itself)."""
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 96
    log("integrate fuse-twice 96^3")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s)
        vid = ctx.volume(gid, (0, 0, 0), (96, 96, 96))
        d, c = seq.frame(5)
        ctx.integrate(t(d), t(c), seq.poses[5], seq.K.as_array())
        F1, W1, C1 = ctx.read_volume(vid)
        ctx.integrate(t(d), t(c), seq.poses[5], seq.K.as_array())
        F2, W2, C2 = ctx.read_volume(vid)
        np.testing.assert_array_equal(W2, 2 * W1)
        np.testing.assert_array_equal(F2.view(np.uint32), F1.view(np.uint32))
        np.testing.assert_array_equal(C2[..., :3], C1[..., :3])


def test_tiled_equals_single_on_gpu(mvf):
    """The paper's invariant on the device: 2x2x2 subvolumes of 33^3 at
    offsets {0, 31} (two shared voxel layers) hold exactly the voxels of one
    64^3 volume."""
    seq = S.small_room_sequence(seed=1)
    n = 64
    origin, s = (-1.0, -1.0, -1.0), 2.0 / n
    log("integrate tiled vs single 64^3 on device")
    with mvf.Context() as ctx:
        g1 = ctx.grid(origin, s)
        big = ctx.volume(g1, (0, 0, 0), (n, n, n), stream_id=0)
        half = n // 2
        tiles = [(ctx.volume(g1, (ox, oy, oz), (half + 1,) * 3, stream_id=1), (ox, oy, oz))
                 for oz in (0, half - 1) for oy in (0, half - 1) for ox in (0, half - 1)]
        K = seq.K.as_array()
        for i in range(10):
            d, c = seq.frame(i)
            ctx.integrate(t(d), t(c), seq.poses[i], K, stream_id=0)
            ctx.integrate(t(d), t(c), seq.poses[i], K, stream_id=1)
        Fb, Wb, Cb = ctx.read_volume(big)
        for vid, (ox, oy, oz) in tiles:
            F, W, Cc = ctx.read_volume(vid)
            sl = np.s_[oz:oz + half + 1, oy:oy + half + 1, ox:ox + half + 1]
            np.testing.assert_array_equal(W, Wb[sl])
            np.testing.assert_array_equal(F.view(np.uint32), Fb[sl].view(np.uint32))
            np.testing.assert_array_equal(Cc, Cb[sl])


def test_large_room_512_full_volume(mvf):
    """At the KinectFusion-scale size: a 512^3 volume over 3 m (5.86 mm
    voxels), 640x480 frames of the 12-object room; three frames fused on the
    device and in the oracle, every voxel compared."""
    seq = S.large_room_sequence(seed=2, n_frames=300)
    n = 512
    origin, s = (-1.5, -1.5, -1.5), 3.0 / n
    og = O.OGrid(origin, s, 4.0, 128)
    log("integrate 512^3 large room, frames 0, 150, 299")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        ids, ovs = fuse_both(ctx, gid, og, [((0, 0, 0), (n, n, n))], seq, [0, 150, 299])
        _, W, _, err = compare_volume(ctx, ids[0], ovs[0])
        log(f"512^3 ok: observed {(W > 0).sum()} voxels, max |dF| {err:.2e}")


@pytest.mark.parametrize("plane_z", [2.0, 5.0])
def test_far_plane_every_voxel(mvf, plane_z):
    """A volume wholly in view in front of a fronto-parallel plane (the
    roofline probe's geometry, small): at 5 m every voxel lies more than mu
    in front of the plane, so whole bricks take the update with phi = 1
    without their own projection; at 2.0 m the plane cuts the far end of
    the volume (colour band, negative side, unobserved voxels behind).  Both
    equal the oracle: W and colour bit-exact, F within 1e-5."""
    n = 72
    s = 0.01
    origin = (-0.36, -0.36, 1.5)
    K = np.array([300.0, 300.0, 159.5, 119.5], np.float32)
    T = np.zeros((3, 4))
    T[:, :3] = np.eye(3)
    depth = np.full((240, 320), plane_z, np.float32)
    depth[:3, :] = 0.0                      # a few invalid rows at the top
    rgb = np.zeros((240, 320, 3), np.uint8)
    rgb[..., 0] = 200
    og = O.OGrid(origin, s, 4.0, 128)
    log(f"far plane z={plane_z}, {n}^3")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        vid = ctx.volume(gid, (0, 0, 0), (n, n, n))
        ov = O.OVolume.empty((n, n, n))
        for k in range(3):
            O.integrate(ov, og, depth, rgb, K, T)
            ctx.integrate(t(depth), t(rgb), T, K)
        F, W, Cc = ctx.read_volume(vid)
        st = ctx.stats()
        np.testing.assert_array_equal(W, ov.W)
        np.testing.assert_array_equal(Cc, ov.Cc)
        assert np.abs(F.astype(np.float64) - ov.F).max() <= 1e-5
        # the counters: every update counted once, each brick in at most one class
        assert st["voxels_updated"] == int(ov.W.sum())
        nb = (n // 8) ** 3
        assert st["bricks_projected"] + st["bricks_deep"] <= 3 * nb
        if plane_z > 4:
            assert int((W == 3).sum()) > 0.9 * n ** 3
            # bricks under the invalid top rows are visited, the rest deep
            assert st["bricks_deep"] > 0.8 * 3 * nb, st
        else:
            assert st["bricks_projected"] > 0 and st["bricks_deep"] > 0, st
