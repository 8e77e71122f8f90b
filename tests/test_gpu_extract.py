"""Surface points on the device (mvf_volume_extract) against the oracle's
extraction of the same volume state (Input and Output: V and N, at most one
vertex per voxel; Metrics; Insertion and Removal).

The oracle reads the device's own binary32 TSDF and weights, so the choice
of emitting voxels and edges is taken on the same values: the point count
and the set of emitting voxels must agree exactly, positions within 1e-4 m
(binary32 against binary64 arithmetic on the same corners: a few 1e-7 m in
practice) and unit normals within 2e-3.  The device writes in brick order,
the oracle in voxel order; both are sorted by global voxel before the
comparison."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S
from tests.util import fuse_both, log, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


def _sorted(G, *arrs):
    order = np.lexsort((G[:, 0], G[:, 1], G[:, 2]))
    return [G[order]] + [a[order] for a in arrs]


def _check(ctx, vid, og, offset, dims):
    F, W, _ = ctx.read_volume(vid)
    ov = O.OVolume(dims, offset, F.astype(np.float64), W, np.zeros(W.shape + (4,), np.uint8))
    ref = O.extract(ov, og, F32=F)
    got = ctx.extract(vid)
    assert got["n"] == ref["n"], f"device {got['n']} points, oracle {ref['n']}"
    assert got["n"] <= int(np.prod(dims))
    if got["n"] == 0:
        return 0
    Gd, Vd, Nd = _sorted(got["G"].cpu().numpy(), got["V"].cpu().numpy().astype(np.float64),
                         got["N"].cpu().numpy().astype(np.float64))
    Go, Vo, No = _sorted(ref["G"], ref["V"], ref["N"])
    np.testing.assert_array_equal(Gd, Go)
    dv = np.abs(Vd - Vo).max()
    assert dv <= 1e-4, f"max |dV| = {dv}"
    ok = np.isfinite(No).all(axis=1)
    assert np.array_equal(ok, np.isfinite(Nd).all(axis=1))
    dn = np.abs(Nd[ok] - No[ok]).max() if ok.any() else 0.0
    assert dn <= 2e-3, f"max |dN| = {dn}"
    return got["n"]


def test_small_room_128_points(mvf):
    """The 128^3 small-room volume after its ten 320x240 frames."""
    log("extract 128^3 small room")
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 128
    og = O.OGrid(origin, s, 4.0, 128)
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        ids, _ = fuse_both(ctx, gid, og, [((0, 0, 0), (128, 128, 128))], seq, range(10))
        n = _check(ctx, ids[0], og, (0, 0, 0), (128, 128, 128))
        assert n > 3000
        log(f"small room: {n} points")


@pytest.mark.parametrize("seed", range(4))
def test_ragged_offset_volumes(mvf, seed):
    """Volumes whose dims are not multiples of the 8-voxel brick, at
    non-zero global offsets, several of them on one grid (the points of each
    come from its own voxels only)."""
    rng = np.random.default_rng(700 + seed)
    seq = S.small_room_sequence(seed=1)
    n = 96
    origin, s = (-1.0, -1.0, -1.0), 2.0 / n
    og = O.OGrid(origin, s, 4.0, 128)
    specs = []
    for _ in range(3):
        dims = tuple(int(x) for x in rng.integers(9, 61, 3))
        off = tuple(int(x) for x in rng.integers(0, n - 9, 3))
        specs.append((off, dims))
    log(f"extract ragged seed={seed} {specs}")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        ids, _ = fuse_both(ctx, gid, og, specs, seq, range(0, 10, 2))
        for vid, (off, dims) in zip(ids, specs):
            _check(ctx, vid, og, off, dims)


def test_capacity_prefix_swap_and_empty(mvf):
    """A capacity below the total writes the first points of the full
    output; a swapped-out volume gives the same points as before; a volume
    that was never observed gives none."""
    import torch
    seq = S.small_room_sequence(seed=1)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 64
    og = O.OGrid(origin, s, 4.0, 128)
    log("extract capacity / swap / empty")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        ids, _ = fuse_both(ctx, gid, og, [((0, 0, 0), (64, 64, 64))], seq, range(10))
        empty = ctx.volume(gid, (64, 0, 0), (16, 16, 16))
        full = ctx.extract(ids[0])
        k = full["n"] // 3
        V = torch.empty((k, 3), dtype=torch.float32, device="cuda")
        N = torch.empty((k, 3), dtype=torch.float32, device="cuda")
        import ctypes as C
        n = C.c_int64()
        from paper_1511_07106_amd import _lib as L
        L.check(ctx.lib.mvf_volume_extract(ctx.h, ids[0], C.c_void_p(V.data_ptr()), C.c_void_p(N.data_ptr()),
                                           None, k, C.byref(n), None), "mvf_volume_extract")
        assert n.value == full["n"]
        assert torch.equal(V, full["V"][:k]) and torch.equal(N, full["N"][:k])
        ctx.swap_out(ids[0])
        assert not ctx.query(ids[0])[0]
        again = ctx.extract(ids[0])
        assert torch.equal(again["V"], full["V"]) and torch.equal(again["G"], full["G"])
        assert ctx.extract(empty)["n"] == 0


def test_large_room_512_points(mvf):
    """The 512^3 large-room volume (3 m, 5.86 mm voxels) after three 640x480
    frames."""
    seq = S.large_room_sequence(seed=2)
    K = seq.K.as_array()
    n = 512
    origin, s = (-1.5, -1.5, -1.5), 3.0 / n
    og = O.OGrid(origin, s, 4.0, 128)
    log("extract 512^3 large room, 3 frames")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, s, 4.0, 128)
        vid = ctx.volume(gid, (0, 0, 0), (n, n, n))
        for i, (d, c) in zip((0, 1, 2), seq.frames([0, 1, 2], threads=16)):
            ctx.integrate(t(d), t(c), seq.poses[i], K)
        m = _check(ctx, vid, og, (0, 0, 0), (n, n, n))
        assert m > 20000
        log(f"large room: {m} points")
