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


def test_step_mixed_image_sizes_equals_plain(mvf):
    """Streams of different, ragged image sizes in one step (frame
    preparation runs over the largest image and each stream masks its own
    bounds; its items are read from the step's host slot): the same bits as
    the plain calls."""
    import torch
    sizes = [(160, 120), (97, 61), (128, 96)]
    seqs = []
    for i, (w, h) in enumerate(sizes):
        K = S.Intrinsics(w * 0.82, w * 0.82, (w - 1) / 2, (h - 1) / 2, w, h)
        seqs.append(S.small_room_sequence(seed=2000 + i, n_frames=8, K=K))
    # a lattice over the whole 4 m room, so that the volumes hold wall and
    # sphere surfaces in most frames
    layouts = [[((0, 0, 0), (57, 40, 57))], [((5, 3, 9), (33, 57, 40)), ((30, 0, 0), (24, 24, 33))],
               [((10, 10, 0), (40, 33, 57))]]
    origin, s = (-2.2, -2.2, -2.2), 4.4 / 64
    log("batched step vs plain, mixed image sizes")
    res = []
    for batched in (False, True):
        with mvf.Context() as ctx:
            gid = ctx.grid(origin, s)
            ids = [[ctx.volume(gid, off, dims, stream_id=i) for off, dims in layouts[i]] for i in range(len(seqs))]
            maps = []
            for f in range(0, 8, 2):
                frames, outs = [], []
                for i, seq in enumerate(seqs):
                    d, c = seq.frame(f)
                    frames.append((i, t(d), t(c), seq.poses[f], seq.K.as_array()))
                if batched:
                    outs = [{"depth": torch.empty((h, w), device="cuda"),
                             "vertex": torch.empty((h, w, 3), device="cuda"),
                             "normal": torch.empty((h, w, 3), device="cuda"),
                             "hit": torch.empty((h, w), dtype=torch.int32, device="cuda")} for w, h in sizes]
                    ctx.step(frames, outs)
                else:
                    for (sid, d, c, T, KK), (w, h) in zip(frames, sizes):
                        ctx.integrate(d, c, T, KK, stream_id=sid)
                        outs.append(ctx.raycast(T, KK, w, h, stream_id=sid))
                maps.append([{k: v.cpu().numpy() for k, v in o.items()} for o in outs])
            vols = [[ctx.read_volume(v) for v in per] for per in ids]
            st = ctx.stats()
            res.append((maps, vols, st))
    (m0, v0, s0), (m1, v1, s1) = res
    assert s1["step_launches"] == 4 and s0["voxels_updated"] == s1["voxels_updated"] > 0
    assert all(int((W > 0).sum()) > 0 for per in v1 for _, W, _ in per)
    for a, b in zip(v0, v1):
        for x, y in zip(a, b):
            for p, q in zip(x, y):
                np.testing.assert_array_equal(p.view(np.uint8), q.view(np.uint8))
    assert sum(int((a["hit"] >= 0).sum()) for fa in m0 for a in fa) > 1000
    for fa, fb in zip(m0, m1):
        for a, b in zip(fa, fb):
            for k in a:
                np.testing.assert_array_equal(a[k].view(np.uint8), b[k].view(np.uint8))


def _run_steps(mvf, seqs, layouts, n_frames, configure=None):
    import torch
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 64
    K = seqs[0].K.as_array()
    w, h = seqs[0].K.width, seqs[0].K.height
    n = len(seqs)
    with mvf.Context() as ctx:
        if configure:
            configure(ctx)
        gid = ctx.grid(origin, s)
        ids = [[ctx.volume(gid, off, dims, stream_id=i) for off, dims in layouts[i]] for i in range(n)]
        maps, scheds = [], []
        rendered = {}
        for f in range(n_frames):
            frames = []
            for i, seq in enumerate(seqs):
                if (i, f % 12) not in rendered:
                    rendered[(i, f % 12)] = seq.frame(f % 12)
                d, c = rendered[(i, f % 12)]
                frames.append((i, t(d), t(c), seq.poses[f % 12], K))
            outs = [{"depth": torch.empty((h, w), device="cuda"), "vertex": torch.empty((h, w, 3), device="cuda"),
                     "normal": torch.empty((h, w, 3), device="cuda"),
                     "hit": torch.empty((h, w), dtype=torch.int32, device="cuda")} for _ in range(n)]
            ctx.step(frames, outs)
            scheds.append(ctx.schedule())
            maps.append([{k: v.cpu().numpy() for k, v in o.items()} for o in outs])
        vols = [[ctx.read_volume(v) for v in per] for per in ids]
    return maps, vols, scheds


def _assert_same(a, b):
    (m0, v0, _), (m1, v1, _) = a, b
    for x, y in zip(v0, v1):
        for p, q in zip(x, y):
            for u, v in zip(p, q):
                np.testing.assert_array_equal(u.view(np.uint8), v.view(np.uint8))
    for fa, fb in zip(m0, m1):
        for x, y in zip(fa, fb):
            for k in x:
                np.testing.assert_array_equal(x[k].view(np.uint8), y[k].view(np.uint8))


@pytest.mark.parametrize("sched", [(1, 0, 4), (2, 1, 4), (8, 0, 4), (8, 1, 2), (4, 1, 8)])
def test_every_schedule_gives_the_same_bits(mvf, sched):
    """Schedules change the work decomposition only: z chunk, integration
    grid and lanes per ray leave every output and voxel bit-identical."""
    seqs, layouts = _scenes(3)
    log(f"schedule {sched} vs default")
    ref = _run_steps(mvf, seqs, layouts, 6)
    got = _run_steps(mvf, seqs, layouts, 6, lambda ctx: ctx.set_schedule(*sched))
    assert all(s == {"zchunk": sched[0], "persistent": sched[1], "ray_lanes": sched[2]} for s in got[2])
    _assert_same(ref, got)


def test_autotune_tunes_caches_and_keeps_results(mvf, tmp_path):
    """TUNE mode runs blocks of eight steps on the first steps of a new shape,
    the default schedule between each two of the other candidates, keeps the
    fastest relative to the default blocks around it and appends it to the
    cache; CACHED mode reads it back.  Results equal the default schedule's
    throughout."""
    seqs, layouts = _scenes(2)
    path = str(tmp_path / "tune.jsonl")
    log("autotune: 15 blocks x 8 runs + 4 steps")
    ref = _run_steps(mvf, seqs, layouts, 124)
    got = _run_steps(mvf, seqs, layouts, 124, lambda ctx: ctx.autotune("tune", path))
    _assert_same(ref, got)
    lines = open(path).read().strip().splitlines()
    assert len(lines) == 1
    import json
    rec = json.loads(lines[0])
    chosen = {k: rec[k] for k in ("zchunk", "persistent", "ray_lanes")}
    assert rec["ms"] > 0
    # the tuning steps alternated the default with the others, then the
    # chosen one stays
    default = {"zchunk": 4, "persistent": 0, "ray_lanes": 4}
    assert all(got[2][8 * b] == default for b in range(0, 15, 2))
    assert got[2][8] == {"zchunk": 2, "persistent": 0, "ray_lanes": 4}
    assert got[2][112] == default and got[2][104] == {"zchunk": 4, "persistent": 0, "ray_lanes": 8}
    assert all(s == chosen for s in got[2][120:])
    cached = _run_steps(mvf, seqs, layouts, 2, lambda ctx: ctx.autotune("cached", path))
    assert all(s == chosen for s in cached[2])
    assert len(open(path).read().strip().splitlines()) == 1


def test_autotune_rejects_bad_arguments(mvf, tmp_path):
    """Errors of the schedule API: an unknown mode, a cache line that does
    not parse, a schedule outside the lists."""
    from paper_1511_07106_amd import _lib as L
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"key": "n1:", "zchunk": 4}\n')
    out_of_range = tmp_path / "range.jsonl"
    out_of_range.write_text('{"key": "n1:", "zchunk": 3, "persistent": 0, "ray_lanes": 4, "ms": 1.0}\n')
    with mvf.Context() as ctx:
        for call in (lambda: ctx.lib.mvf_autotune(ctx.h, 7, None),
                     lambda: ctx.lib.mvf_autotune(ctx.h, 1, str(bad).encode()),
                     lambda: ctx.lib.mvf_autotune(ctx.h, 2, str(out_of_range).encode())):
            assert call() == L.MVF_ERR_INVALID_ARG
        with pytest.raises(L.MvfError):
            ctx.set_schedule(3, 0, 4)
        with pytest.raises(L.MvfError):
            ctx.set_schedule(4, 0, 16)
        ctx.autotune("cached", str(tmp_path / "missing.jsonl"))   # a missing file is an empty cache
        assert ctx.schedule() == {"zchunk": 4, "persistent": 0, "ray_lanes": 4}
