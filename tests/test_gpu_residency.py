"""Memory passing (the paper's upload/download of subvolumes) as identities:
swapping a volume out and in, or running under a device budget as small as
one volume, changes no bit of any result."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S
from tests.util import log, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


def _tiles(ctx, gid, n, stream_id=0):
    half = n // 2
    return [ctx.volume(gid, (ox, oy, oz), (half + 1,) * 3, stream_id=stream_id)
            for oz in (0, half - 1) for oy in (0, half - 1) for ox in (0, half - 1)]


def test_swap_round_trip(mvf):
    seq = S.small_room_sequence(seed=1)
    K = seq.K.as_array()
    log("swap out / in round trip 64^3")
    with mvf.Context() as ctx:
        gid = ctx.grid((-1.0, -1.0, -1.0), 2.0 / 64)
        vid = ctx.volume(gid, (0, 0, 0), (64, 64, 64))
        for i in range(3):
            d, c = seq.frame(i)
            ctx.integrate(t(d), t(c), seq.poses[i], K)
        F1, W1, C1 = ctx.read_volume(vid)
        flag1, dist1 = ctx.brick_summary(vid)
        assert flag1.any()
        ctx.swap_out(vid)
        resident, nbytes, active = ctx.query(vid)
        assert not resident and active and nbytes >= 64 ** 3 * 10
        F2, W2, C2 = ctx.read_volume(vid)  # read from the host mirror
        np.testing.assert_array_equal(F2.view(np.uint32), F1.view(np.uint32))
        np.testing.assert_array_equal(W2, W1)
        np.testing.assert_array_equal(C2, C1)
        flag2, dist2 = ctx.brick_summary(vid)  # the summaries travel with the slab
        np.testing.assert_array_equal(flag2, flag1)
        np.testing.assert_array_equal(dist2, dist1)
        ctx.swap_in(vid)
        assert ctx.query(vid)[0]
        F3, W3, C3 = ctx.read_volume(vid)
        np.testing.assert_array_equal(F3.view(np.uint32), F1.view(np.uint32))
        np.testing.assert_array_equal(W3, W1)
        flag3, dist3 = ctx.brick_summary(vid)
        np.testing.assert_array_equal(flag3, flag1)
        np.testing.assert_array_equal(dist3, dist1)
        st = ctx.stats()
        assert st["swaps_out"] == 1 and st["swaps_in"] == 1 and st["bytes_h2d"] == nbytes


@pytest.mark.parametrize("n,budget_volumes", [(64, 1), (64, 3), (416, 1), (416, 3)])
def test_budget_identity(mvf, n, budget_volumes):
    """Eight (n/2 + 1)^3 subvolumes fused and raycast with room for only
    `budget_volumes` of them on the device (waves + swaps) give the same bits
    as with no budget.  At n = 416 a slab (209^3, about 93 MB) is copied in
    two chunks, and a swap-in into the slab of the volume just swapped out
    overlaps that volume's download chunk by chunk."""
    seq = S.small_room_sequence(seed=1)
    K = seq.K.as_array()
    origin, s = (-1.0, -1.0, -1.0), 2.0 / n
    log(f"budget identity, n {n}, room for {budget_volumes} of 8 volumes")
    results = []
    for limited in (False, True):
        with mvf.Context() as ctx:
            gid = ctx.grid(origin, s)
            ids = _tiles(ctx, gid, n)
            if limited:
                ctx.set_budget(budget_volumes * ctx.query(ids[0])[1])
            maps = []
            for i in range(10):
                d, c = seq.frame(i)
                ctx.integrate(t(d), t(c), seq.poses[i], K)
                if i % 3 == 0:
                    out = ctx.raycast(seq.poses[i], K, 320, 240)
                    maps.append({k: v.cpu().numpy() for k, v in out.items()})
            vols = [ctx.read_volume(v) for v in ids]
            st = ctx.stats()
            results.append((maps, vols, st))
    (m0, v0, s0), (m1, v1, s1) = results
    assert s0["swaps_out"] == 0 and s1["swaps_out"] > 0 and s1["swaps_in"] > 0
    for a, b in zip(v0, v1):
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.view(np.uint8), y.view(np.uint8))
    for a, b in zip(m0, m1):
        for k in a:
            np.testing.assert_array_equal(a[k].view(np.uint8), b[k].view(np.uint8))


def test_budget_smaller_than_one_volume_is_an_error(mvf):
    seq = S.small_room_sequence(seed=1)
    log("budget below one volume")
    with mvf.Context(budget_bytes=1 << 20) as ctx:
        gid = ctx.grid((-1.0, -1.0, -1.0), 2.0 / 64)
        ctx.volume(gid, (0, 0, 0), (64, 64, 64))
        d, c = seq.frame(0)
        with pytest.raises(mvf._lib.MvfError) as e:
            ctx.integrate(t(d), t(c), seq.poses[0], seq.K.as_array())
        assert e.value.status == mvf._lib.MVF_ERR_BUDGET


def test_write_read_checkpoint(mvf):
    """mvf_volume_write then mvf_volume_read restores the canonical state
    (F of unobserved voxels reads as 0), through a swap as well."""
    rng = np.random.default_rng(7)
    dims = (21, 13, 30)
    log("write/read checkpoint ragged volume")
    with mvf.Context() as ctx:
        gid = ctx.grid((0, 0, 0), 0.02)
        vid = ctx.volume(gid, (5, -3, 2), dims)
        nz, ny, nx = dims[2], dims[1], dims[0]
        F = rng.uniform(-1, 1, (nz, ny, nx)).astype(np.float32)
        W = rng.integers(0, 5, (nz, ny, nx)).astype(np.uint16)
        Cc = rng.integers(0, 256, (nz, ny, nx, 4)).astype(np.uint8)
        ctx.write_volume(vid, F, W, Cc)
        for swap in (False, True):
            if swap:
                ctx.swap_out(vid)
            F2, W2, C2 = ctx.read_volume(vid)
            np.testing.assert_array_equal(W2, W)
            np.testing.assert_array_equal(F2, np.where(W > 0, F, 0))
            np.testing.assert_array_equal(C2, Cc)


def test_evict_keeps_state_and_stops_updates(mvf):
    """An evicted volume (removed from H) keeps its state and is no longer
    integrated; placing it again resumes fusion."""
    seq = S.small_room_sequence(seed=1)
    K = seq.K.as_array()
    log("evict / place")
    with mvf.Context() as ctx:
        gid = ctx.grid((-1.0, -1.0, -1.0), 2.0 / 48)
        vid = ctx.volume(gid, (0, 0, 0), (48, 48, 48))
        d, c = seq.frame(0)
        ctx.integrate(t(d), t(c), seq.poses[0], K)
        F1, W1, _ = ctx.read_volume(vid)
        ctx.evict(vid, swap_out=True)
        ctx.integrate(t(d), t(c), seq.poses[0], K)
        F2, W2, _ = ctx.read_volume(vid)
        np.testing.assert_array_equal(W2, W1)
        ctx.place(vid)
        ctx.integrate(t(d), t(c), seq.poses[0], K)
        _, W3, _ = ctx.read_volume(vid)
        np.testing.assert_array_equal(W3, 2 * W1)
