"""The largest volume the library takes: 2^30 padded voxels (1024^3: 4 GiB
of F, 2 GiB of W, 4 GiB of colour; every element and byte offset of a plane
still fits the 32-bit addressing), fused from large-room frames and compared
with the oracle on 64^3 windows of it, among them the observed window with
the largest brick indices; volumes beyond the limit are refused.

Voxel values depend only on a voxel's global lattice position, so a window
integrated by the oracle as a volume of its own must equal the same voxels
of the large one (W and colour bit-exact, F within 1e-5)."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S
from tests.util import log, t

pytestmark = pytest.mark.gpu

N = 1024
EXTENT = 6.0
WIN = 64


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


def test_limit_refused(mvf):
    with mvf.Context() as ctx:
        gid = ctx.grid((-EXTENT / 2,) * 3, EXTENT / N)
        with pytest.raises(mvf._lib.MvfError):
            ctx.volume(gid, (0, 0, 0), (N + 1, N, N))      # pads to 1032 x 1024 x 1024 > 2^30
        with pytest.raises(mvf._lib.MvfError):
            ctx.volume(gid, (0, 0, 0), (2049, 8, 8))
        ctx.volume(gid, (0, 0, 0), (N, N, N))              # exactly 2^30: accepted (not resident yet)


def test_max_volume_windows_vs_oracle(mvf):
    seq = S.large_room_sequence(seed=2, n_frames=5)
    K = seq.K.as_array()
    ids = [0, 2, 4]
    frames = seq.frames(ids, threads=16)
    origin = (-EXTENT / 2,) * 3
    og = O.OGrid(origin, EXTENT / N, 4.0, 128)
    log("1024^3 volume: integrate 3 large-room frames")
    with mvf.Context() as ctx:
        gid = ctx.grid(origin, EXTENT / N, 4.0, 128)
        vid = ctx.volume(gid, (0, 0, 0), (N, N, N))
        for i, (d, c) in zip(ids, frames):
            ctx.integrate(t(d), t(c), seq.poses[i], K)
        st = ctx.stats()
        F, W, Cc = ctx.read_volume(vid)
    assert st["voxels_updated"] == int(W.sum(dtype=np.int64))
    # 64^3 windows on a 16^3 grid: the one with the most band voxels, and the
    # observed one with the largest offsets (the far corner of the planes)
    band = (W > 0) & (np.abs(F) < 1.0)
    nb = N // WIN
    counts = band.reshape(nb, WIN, nb, WIN, nb, WIN).sum(axis=(1, 3, 5))   # (z, y, x) blocks
    obs = (W > 0).reshape(nb, WIN, nb, WIN, nb, WIN).sum(axis=(1, 3, 5))
    zb, yb, xb = np.unravel_index(int(np.argmax(counts)), counts.shape)
    windows = [(xb, yb, zb)]
    # brick order is x-major: the largest x block first, then y, then z
    cand = np.argwhere(obs > 1000)
    far = max(cand.tolist(), key=lambda b: (b[2], b[1], b[0]))
    windows.append((far[2], far[1], far[0]))
    assert counts.max() > 1000
    for bx, by, bz in windows:
        off = (int(bx) * WIN, int(by) * WIN, int(bz) * WIN)
        log(f"window at {off}")
        ov = O.OVolume.empty((WIN, WIN, WIN), off)
        for i, (d, c) in zip(ids, frames):
            O.integrate(ov, og, d, c, K, seq.poses[i])
        sl = np.s_[off[2]:off[2] + WIN, off[1]:off[1] + WIN, off[0]:off[0] + WIN]
        np.testing.assert_array_equal(W[sl], ov.W)
        np.testing.assert_array_equal(Cc[sl], ov.Cc)
        err = float(np.abs(F[sl].astype(np.float64) - ov.F).max())
        assert err <= 1e-5, err
        assert int((ov.W > 0).sum()) > 1000
