"""Checkpoint / resume in a new context, and the residency manager's
out-of-memory paths (Memory Passing: volumes are swapped, not lost).

- a context saved mid-sequence and loaded into a fresh context continues
  bit for bit like the original (volume state, raycast maps), with volumes
  that were resident, swapped out and never observed;
- placement state (which cell owns which volume) survives: a corridor walk
  resumed from a checkpoint makes the same insertions and removals;
- an injected failure of a slab allocation is absorbed by dropping the
  slab pool and retrying (results equal an undisturbed run); two failures
  in a row give MVF_ERR_OOM with the context left usable."""
import os
import tempfile

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


def _state(ctx, ids):
    return [ctx.read_volume(v) for v in ids]


def _same(a, b):
    for (F1, W1, C1), (F2, W2, C2) in zip(a, b):
        assert np.array_equal(F1.view(np.uint32), F2.view(np.uint32))
        assert np.array_equal(W1, W2) and np.array_equal(C1, C2)


def test_checkpoint_resume_bit_identical(mvf):
    seq = S.small_room_sequence(seed=1)
    K = seq.K.as_array()
    n = 64
    origin, s = (-1.0, -1.0, -1.0), 2.0 / n
    h = n // 2
    offs = [(0, 0, 0), (h - 1, 0, 0), (0, h - 1, 0), (h - 1, h - 1, 0)]
    frames = [(t(d), t(c)) for d, c in seq.frames(range(10), threads=10)]
    path = os.path.join(tempfile.mkdtemp(), "ckpt.mvf")
    log("checkpoint / resume small room")
    with mvf.Context() as A:
        gid = A.grid(origin, s, 4.0, 128)
        ids = [A.volume(gid, o, (h + 1, h + 1, n)) for o in offs]
        never = A.volume(gid, (0, 0, n + 10), (16, 16, 16))     # out of view: never observed
        A.set_budget(2 * A.query(ids[0])[1])                  # two of four fit: some are swapped out
        for i in range(5):
            A.integrate(*frames[i], seq.poses[i], K)
        A.evict(ids[3])                                       # inactive, state kept
        A.save(path)
        for i in range(5, 10):
            A.integrate(*frames[i], seq.poses[i], K)
        ga = {k: v.cpu().numpy() for k, v in A.raycast(seq.poses[9], K, 320, 240).items()}
        sa = _state(A, ids + [never])
        assert A.stats()["swaps_out"] > 0
    with mvf.Context() as B:
        B.set_budget(2 * (1 << 30))
        B.load(path)
        assert not B.query(ids[3])[2] and B.query(ids[0])[2]
        assert [B.dims(v) for v in ids] == [(h + 1, h + 1, n)] * 4
        for i in range(5, 10):
            B.integrate(*frames[i], seq.poses[i], K)
        gb = {k: v.cpu().numpy() for k, v in B.raycast(seq.poses[9], K, 320, 240).items()}
        sb = _state(B, ids + [never])
    _same(sa, sb)
    assert np.array_equal(ga["hit"], gb["hit"])
    assert np.array_equal(ga["depth"].view(np.uint32), gb["depth"].view(np.uint32))
    assert int((sa[-1][1] > 0).sum()) == 0
    # loading into a used context, or a file that is not a checkpoint
    with mvf.Context() as C:
        C.grid(origin, s)
        with pytest.raises(mvf._lib.MvfError):
            C.load(path)
    bad = path + ".bad"
    with open(bad, "wb") as f:
        f.write(open(path, "rb").read()[:200])
    with mvf.Context() as D:
        with pytest.raises(mvf._lib.MvfError):
            D.load(bad)
        D.load(path)   # the failed load left it empty


def test_checkpoint_keeps_placement(mvf):
    seq = S.corridor_sequence(seed=3, n_frames=2000)
    K = seq.K.as_array()
    classes = [(256, 4), (128, 6)]
    idx = list(range(0, 1200, 60))
    frames = [t(d) for d, _ in seq.frames(idx, threads=16)]
    path = os.path.join(tempfile.mkdtemp(), "ckpt.mvf")
    log("checkpoint / resume corridor placement")

    def walk(ctx, gid, steps):
        out = []
        for j in steps:
            d = frames[j]
            a, r, _ = ctx.placement_update_classes(d, seq.poses[idx[j]], K, gid, classes, 1.5)
            ctx.integrate(d, None, seq.poses[idx[j]], K)
            out.append((sorted(a), sorted(r)))
        return out

    with mvf.Context(budget_bytes=600 << 20) as A:
        gid = A.grid((0.0, -1.0, 0.0), 0.00293, 4.0, 128)
        walk(A, gid, range(10))
        A.save(path)
        rest_a = walk(A, gid, range(10, 20))
        ids_a = [v for v in range(400) if _alive(A, v)]
        sa = _state(A, ids_a)
    with mvf.Context(budget_bytes=600 << 20) as B:
        B.load(path)
        rest_b = walk(B, gid, range(10, 20))
        ids_b = [v for v in range(400) if _alive(B, v)]
        sb = _state(B, ids_b)
    assert rest_a == rest_b and ids_a == ids_b
    assert any(a or r for a, r in rest_a)
    _same(sa, sb)


def _alive(ctx, vid):
    try:
        ctx.describe(vid)
        return True
    except Exception:
        return False


def test_slab_allocation_failure_retry_and_oom(mvf):
    seq = S.small_room_sequence(seed=1)
    K = seq.K.as_array()
    frames = [(t(d), t(c)) for d, c in seq.frames(range(6), threads=6)]
    origin, s = (-1.0, -1.0, -1.0), 2.0 / 96
    # three volumes of different sizes under a budget of two: a new slab is
    # allocated (no pooled slab of its size) after an eviction
    specs = [((0, 0, 0), (50, 96, 96)), ((46, 0, 0), (50, 96, 96)), ((0, 40, 0), (96, 56, 96))]

    def run(fault):
        if fault:
            os.environ["MVF_FAULT_SLAB_ALLOCS"] = str(fault)
        try:
            ctx = mvf.Context()
        finally:
            os.environ.pop("MVF_FAULT_SLAB_ALLOCS", None)
        with ctx:
            gid = ctx.grid(origin, s, 4.0, 128)
            ids = [ctx.volume(gid, o, d) for o, d in specs]
            ctx.set_budget(ctx.query(ids[0])[1] + ctx.query(ids[2])[1] + (1 << 20))
            errors = 0
            for i in range(6):
                try:
                    ctx.integrate(*frames[i], seq.poses[i], K)
                except mvf._lib.MvfError as e:
                    assert e.status == mvf._lib.MVF_ERR_OOM
                    errors += 1
            st = _state(ctx, ids)
            stats = ctx.stats()
        return st, errors, stats

    log("slab allocation failure injection")
    clean, e0, st0 = run(0)
    assert e0 == 0 and st0["swaps_out"] > 0
    retried, e1, _ = run(1)          # the first slab allocation fails once: the retry succeeds
    assert e1 == 0
    _same(clean, retried)
    oom, e2, _ = run(2)              # fails twice: that call reports MVF_ERR_OOM, the rest go on
    assert e2 == 1
    # the other frames were integrated: every volume holds observations
    assert all(int((W > 0).sum()) > 0 for _, W, _ in oom)
