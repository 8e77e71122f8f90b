"""The batched form (one persistent integration launch and one persistent
raycast launch over a device volume table, captured once in a HIP graph and
replayed) gives the same bits as the plain per-volume calls."""
import numpy as np
import pytest

from synth import scenes as S
from tests.util import log, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


def _scenes(n_streams, w=160, h=120):
    K = S.Intrinsics(w * 0.82, w * 0.82, (w - 1) / 2, (h - 1) / 2, w, h)
    seqs = [S.small_room_sequence(seed=1000 + i, n_frames=12, K=K) for i in range(n_streams)]
    rng = np.random.default_rng(42)
    layouts = []
    for i in range(n_streams):
        nv = int(rng.integers(1, 4))
        vols = []
        for _ in range(nv):
            dims = tuple(int(x) for x in rng.choice([24, 33, 40, 57], 3))
            off = tuple(int(x) for x in rng.integers(0, 30, 3))
            vols.append((off, dims))
        layouts.append(vols)
    return seqs, layouts


@pytest.mark.parametrize("n_streams", [1, 5])
def test_step_equals_plain(mvf, n_streams):
    seqs, layouts = _scenes(n_streams)
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 64
    K = seqs[0].K.as_array()
    w, h = seqs[0].K.width, seqs[0].K.height
    log(f"batched step vs plain, {n_streams} streams")
    import torch
    res = []
    for batched in (False, True):
        with mvf.Context() as ctx:
            gid = ctx.grid(origin, s)
            ids = [[ctx.volume(gid, off, dims, stream_id=i) for off, dims in layouts[i]]
                   for i in range(n_streams)]
            maps = []
            for f in range(0, 12, 2):
                frames, outs = [], []
                for i, seq in enumerate(seqs):
                    d, c = seq.frame(f)
                    frames.append((i, t(d), t(c), seq.poses[f], K))
                if batched:
                    outs = [{"depth": torch.empty((h, w), device="cuda"),
                             "vertex": torch.empty((h, w, 3), device="cuda"),
                             "normal": torch.empty((h, w, 3), device="cuda"),
                             "hit": torch.empty((h, w), dtype=torch.int32, device="cuda")}
                            for _ in range(n_streams)]
                    ctx.step(frames, outs)
                else:
                    for (sid, d, c, T, KK) in frames:
                        ctx.integrate(d, c, T, KK, stream_id=sid)
                        outs.append(ctx.raycast(T, KK, w, h, stream_id=sid))
                maps.append([{k: v.cpu().numpy() for k, v in o.items()} for o in outs])
            vols = [[ctx.read_volume(v) for v in per] for per in ids]
            st = ctx.stats()
            res.append((maps, vols, st))
    (m0, v0, s0), (m1, v1, s1) = res
    assert s1["step_launches"] == 6 and s0["step_launches"] == 0
    assert s0["voxels_updated"] == s1["voxels_updated"] > 0
    for a, b in zip(v0, v1):
        for x, y in zip(a, b):
            for p, q in zip(x, y):
                np.testing.assert_array_equal(p.view(np.uint8), q.view(np.uint8))
    for fa, fb in zip(m0, m1):
        for a, b in zip(fa, fb):
            for k in a:
                np.testing.assert_array_equal(a[k].view(np.uint8), b[k].view(np.uint8))
