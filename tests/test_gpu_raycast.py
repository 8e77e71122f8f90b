"""GPU parity of the multi-volume raycast against the CPU oracle (validity
and hit volume exact, depth within 1e-4 m)."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S
from tests.util import check_raycast, compare_volume, fuse_both, log, raycast_both, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


def _lattice(og, dims, off):
    nx, ny, nz = dims
    gz, gy, gx = np.meshgrid(np.arange(nz) + off[2], np.arange(ny) + off[1], np.arange(nx) + off[0],
                             indexing="ij")
    s = og.voxel_size
    return np.stack([og.origin[0] + s * (gx + 0.5), og.origin[1] + s * (gy + 0.5),
                     og.origin[2] + s * (gz + 0.5)], -1)


def test_small_room_raycast_same_volume(mvf):
    """Fuse 10 frames in the oracle, load that volume onto the device, and
    raycast the last pose and a held-out pose on both sides."""
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 128
    og = O.OGrid(origin, s, 4.0, 128)
    ov = O.OVolume.empty((128, 128, 128))
    K = seq.K.as_array()
    for i in range(10):
        d, c = seq.frame(i)
        O.integrate(ov, og, d, c, K, seq.poses[i])
    held_out = S.look_at([0.7, -0.6, 0.25], [0.0, 0.05, -0.1])
    log("raycast 128^3 small room (oracle-fused volume)")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        vid = ctx.volume(gid, (0, 0, 0), (128, 128, 128))
        ctx.write_volume(vid, ov.F32(), ov.W, ov.Cc)
        for T in (seq.poses[9], held_out):
            g, rc = raycast_both(ctx, [ov], og, K, T, 320, 240)
            n = check_raycast(g, rc, [vid])
            assert n > 10000


def test_small_room_end_to_end(mvf):
    """Integration and raycast both on the device vs both in the oracle:
    pixels whose march saw a near-zero sign test are excluded (the TSDFs
    agree only to 1e-5)."""
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 128
    og = O.OGrid(origin, s, 4.0, 128)
    K = seq.K.as_array()
    log("integrate + raycast end to end 128^3")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        ids, ovs = fuse_both(ctx, gid, og, [((0, 0, 0), (128, 128, 128))], seq, range(10))
        g, rc = raycast_both(ctx, ovs, og, K, seq.poses[9], 320, 240)
        amb = rc["ambiguous"].astype(bool)
        print(f"[parity] small room 128^3 end to end: ambiguous fraction {amb.mean():.2e}", flush=True)
        # measured 2.6e-5 on this scene; the parity bar for end-to-end maps is 1e-4
        assert amb.mean() < 1e-4
        hit_g, hit_o = g["hit"] >= 0, rc["hit"] >= 0
        np.testing.assert_array_equal(hit_g[~amb], hit_o[~amb])
        both = hit_g & hit_o & ~amb
        dd = np.abs(g["depth"].astype(np.float64) - rc["depth"])[both]
        assert dd.max() <= 1e-4, dd.max()


@pytest.mark.parametrize("seed", range(4))
def test_random_fields_multi_volume(mvf, seed):
    """Several ragged volumes at different offsets on one grid, filled with
    random smooth fields and random unobserved holes; random camera and
    image sizes (not multiples of the 16x16 tile)."""
    rng = np.random.default_rng(200 + seed)
    s = 1.0 / 32
    origin = (-1.0, -1.0, -1.0)
    og = O.OGrid(origin, s, 4.0)
    nvol = int(rng.integers(1, 5))
    specs = []
    for _ in range(nvol):
        dims = tuple(int(x) for x in rng.integers(5, 45, 3))
        off = tuple(int(x) for x in rng.integers(0, 30, 3))
        specs.append((off, dims))
    c = rng.uniform(-0.2, 0.6, 3)
    r = rng.uniform(0.2, 0.5)
    wv = rng.normal(size=3)
    ovs = []
    for off, dims in specs:
        ov = O.OVolume.empty(dims, off)
        x = _lattice(og, dims, off)
        f = (np.linalg.norm(x - c, axis=-1) - r) / og.mu + 0.3 * np.sin(x @ wv * 4)
        ov.F[:] = np.clip(f, -1, 1)
        ov.W[:] = 1 + rng.integers(0, 3, ov.W.shape)
        holes = rng.uniform(size=ov.W.shape) < 0.02
        ov.W[holes] = 0
        ov.F[holes] = 0.0
        ovs.append(ov)
    w, h = int(rng.integers(20, 130)), int(rng.integers(20, 100))
    K = np.array([w * 0.8, w * 0.8, (w - 1) / 2, (h - 1) / 2], np.float32)
    T = S.look_at(c + rng.normal(size=3) * 0.3 + np.array([0, 0, 1.5]), c, up=(0, 1, 0))
    log(f"raycast random fields seed={seed} nvol={nvol} img={w}x{h}")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0)
        ids = []
        for (off, dims), ov in zip(specs, ovs):
            vid = ctx.volume(gid, off, dims)
            ctx.write_volume(vid, ov.F32(), ov.W, ov.Cc)
            ids.append(vid)
        g, rc = raycast_both(ctx, ovs, og, K, T, w, h)
        check_raycast(g, rc, ids)


def test_no_volumes_writes_no_hits(mvf):
    log("raycast with no active volume")
    with mvf.Context() as ctx:
        ctx.grid((0, 0, 0), 0.01)
        out = ctx.raycast(S.look_at([0, 0, -1], [0, 0, 0]), [50, 50, 20, 15], 40, 30)
        import torch
        torch.cuda.synchronize()
        assert (out["depth"] == 0).all() and (out["hit"] == -1).all()
        assert torch.isnan(out["normal"]).all()


def test_tiled_equals_single_raycast_on_gpu(mvf):
    """Raycast of 8 overlapping subvolumes equals the single volume's maps
    bit for bit on the device (Comparison to KinectFusion)."""
    seq = S.small_room_sequence(seed=1)
    n = 64
    origin, s = (-1.0, -1.0, -1.0), 2.0 / n
    K = seq.K.as_array()
    log("raycast tiled vs single 64^3 on device")
    with mvf.Context() as ctx:
        g1 = ctx.grid(origin, s)
        ctx.volume(g1, (0, 0, 0), (n, n, n), stream_id=0)
        half = n // 2
        for oz in (0, half - 1):
            for oy in (0, half - 1):
                for ox in (0, half - 1):
                    ctx.volume(g1, (ox, oy, oz), (half + 1,) * 3, stream_id=1)
        for i in range(10):
            d, c = seq.frame(i)
            ctx.integrate(t(d), t(c), seq.poses[i], K, stream_id=0)
            ctx.integrate(t(d), t(c), seq.poses[i], K, stream_id=1)
        for T in (seq.poses[9], seq.poses[4]):
            a = ctx.raycast(T, K, 320, 240, stream_id=0)
            b = ctx.raycast(T, K, 320, 240, stream_id=1)
            import torch
            torch.cuda.synchronize()
            assert (a["depth"] > 0).float().mean() > 0.2
            for key in ("depth", "vertex", "normal"):
                x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
                np.testing.assert_array_equal(x.view(np.uint32), y.view(np.uint32))


def test_large_room_512_sampled_rays(mvf):
    """512^3 at full frame size (640x480): the oracle-fused volume from 3
    frames, raycast on the device in the launch shape the benchmark uses,
    every pixel compared."""
    seq = S.large_room_sequence(seed=2, n_frames=300)
    n = 512
    origin, s = (-1.5, -1.5, -1.5), 3.0 / n
    og = O.OGrid(origin, s, 4.0, 128)
    ov = O.OVolume.empty((n, n, n))
    K = seq.K.as_array()
    for i in (0, 150, 299):
        d, c = seq.frame(i)
        O.integrate(ov, og, d, c, K, seq.poses[i])
    log("raycast 512^3 large room 640x480")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        vid = ctx.volume(gid, (0, 0, 0), (n, n, n))
        F32 = ov.F32()
        ctx.write_volume(vid, F32, ov.W, ov.Cc)
        g, rc = raycast_both(ctx, [ov], og, K, seq.poses[150], 640, 480, F32=[F32])
        nhit = check_raycast(g, rc, [vid])
        log(f"512^3 raycast ok, {nhit} pixels hit")
        assert nhit > 50000
