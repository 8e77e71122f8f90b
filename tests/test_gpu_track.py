"""Camera tracking on the device (mvf_depth_maps, mvf_track) against the
oracle (Depth Map Conversion; Camera Tracking).

The maps and every association decision follow the binary32 contract, so
the vertex and normal maps of each pyramid level are bit-identical and
every Gauss-Newton step pairs exactly the oracle's pixels; the sums are
binary64 in another order (per block, then over blocks), so the squared
error of a step agrees to 1e-9 relative and the final pose to 1e-6."""
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


def _same_nan(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(a[~np.isnan(a)], b[~np.isnan(b)])


@pytest.mark.parametrize("which", ["room", "ragged"])
def test_depth_maps_bit_exact(mvf, which):
    if which == "room":
        seq = S.large_room_sequence(seed=2, n_frames=5)
        d, _ = seq.frame(3)
        K = seq.K.as_array()
    else:
        rng = np.random.default_rng(9)
        h, w = 37, 53
        d = rng.uniform(0.3, 4.0, (h, w)).astype(np.float32)
        d[rng.random((h, w)) < 0.1] = 0.0
        d[rng.random((h, w)) < 0.03] = np.nan
        d[rng.random((h, w)) < 0.03] = np.inf
        d[rng.random((h, w)) < 0.03] = -1.0
        K = np.array([40.0, 41.0, 26.2, 17.9], np.float32)
    log(f"depth maps {which}")
    with mvf.Context() as ctx:
        for smooth in (0.0, 0.09):
            D = O.depth_pyramid(O.depth_smooth(d, smooth) if smooth else d, 3)
            for lvl in range(3):
                V, N = ctx.depth_maps(t(d), K, level=lvl, smooth=smooth)
                Vo, No = O.vertex_normal(D[lvl], O.level_K(K, lvl))
                assert V.shape == Vo.shape
                assert _same_nan(V.cpu().numpy(), Vo) and _same_nan(N.cpu().numpy(), No), (smooth, lvl)


def _fused_model(mvf, ctx, seq, upto, n=512, extent=3.0):
    """A 512^3 volume fused with the true poses of frames 0..upto, and the
    raycast maps at pose `upto` (the model the next frame is tracked
    against)."""
    gid = ctx.grid((-extent / 2,) * 3, extent / n, 4.0, 128)
    ctx.volume(gid, (0, 0, 0), (n, n, n))
    K = seq.K.as_array()
    for i, (d, c) in zip(range(upto + 1), seq.frames(range(upto + 1), threads=16)):
        ctx.integrate(t(d), t(c), seq.poses[i], K)
    return ctx.raycast(seq.poses[upto], K, seq.K.width, seq.K.height)


@pytest.mark.parametrize("frame", [6, 40])
def test_track_matches_oracle_and_truth(mvf, frame):
    """Frame k+1 of the large room tracked against the raycast of a volume
    fused from frames 0..k, from the pose of frame k: every step pairs the
    oracle's pixels, the pose equals the oracle's and lies near the true
    pose of frame k+1."""
    import torch
    seq = S.large_room_sequence(seed=2, n_frames=frame + 2)
    K = seq.K.as_array()
    log(f"track large room frame {frame + 1}")
    with mvf.Context() as ctx:
        model = _fused_model(mvf, ctx, seq, frame)
        torch.cuda.synchronize()
        d, _ = seq.frame(frame + 1)
        T0 = seq.poses[frame]
        T_dev, st = ctx.track(t(d), K, model, T0, T0)
    Vm = model["vertex"].cpu().numpy()
    Nm = model["normal"].cpu().numpy()
    T32 = np.asarray(T0, np.float32).astype(np.float64)
    T_ora, steps = O.icp_track(d, K, Vm, Nm, T32, T0)
    assert [s[1] for s in steps] == st["pairs"]
    for (_, _, e), e_dev in zip(steps, st["sq_err"]):
        assert abs(e - e_dev) <= 1e-9 * max(e, 1e-12)
    assert np.abs(T_dev - T_ora).max() <= 1e-6
    T1 = seq.poses[frame + 1]
    et = np.linalg.norm(T_dev[:, 3] - T1[:, 3])
    R = T_dev[:, :3].T @ T1[:, :3]
    er = np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    e0 = np.linalg.norm(T0[:, 3] - T1[:, 3])
    print(f"[track] frame {frame + 1}: start {1e3 * e0:.2f} mm, tracked {1e3 * et:.2f} mm / {er:.3f} deg, "
          f"pairs {st['pairs'][-1]}", flush=True)
    assert et < 5e-3 and er < 0.3


def test_track_edge_cases(mvf):
    """An empty model or frame leaves the pose as given (no step has 6
    pairs); bad arguments are rejected."""
    import torch
    seq = S.large_room_sequence(seed=2, n_frames=2)
    K = seq.K.as_array()
    d, _ = seq.frame(1)
    H, W = d.shape
    empty = {"vertex": torch.full((H, W, 3), float("nan"), device="cuda"),
             "normal": torch.full((H, W, 3), float("nan"), device="cuda")}
    log("track edge cases")
    with mvf.Context() as ctx:
        T, st = ctx.track(t(d), K, empty, seq.poses[0], seq.poses[1])
        assert np.array_equal(T, seq.poses[1]) and st["pairs"] == [0] * 19
        T, st = ctx.track(t(np.zeros_like(d)), K, empty, seq.poses[0], seq.poses[1], iters=(3,))
        assert np.array_equal(T, seq.poses[1]) and st["pairs"] == [0] * 3
        with pytest.raises(mvf._lib.MvfError):
            ctx.track(t(d), K, empty, seq.poses[0], seq.poses[1], iters=(40, 20, 10))
        small = {"vertex": empty["vertex"][:100], "normal": empty["normal"][:100]}
        with pytest.raises(ValueError):
            ctx.track(t(d), K, small, seq.poses[0], seq.poses[1])
