"""GPU placement (Dynamic Mapping for SLAM): endpoint cell counts equal the
oracle's exactly; the insertion/removal sequence over a corridor walk equals
the oracle policy applied to the oracle counts."""
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


@pytest.mark.parametrize("which", ["room", "corridor"])
def test_counts_match_oracle(mvf, which):
    seq = S.small_room_sequence(seed=1) if which == "room" else S.corridor_sequence(seed=3, n_frames=600)
    frames = [0, 3, 7] if which == "room" else [0, 250, 599]
    s = 0.00293
    og = O.OGrid((0.0, -1.0, 0.0), s)
    log(f"placement counts {which}")
    with mvf.Context() as ctx:
        gid = ctx.grid(og.origin, s)
        for d_v in (66, 256):
            for i in frames:
                d, _ = seq.frame(i)
                a = ctx.placement_count(t(d), seq.poses[i], seq.K.as_array(), gid, d_v)
                b = O.placement_counts(d, seq.K.as_array(), seq.poses[i], og, d_v)
                assert a == b


def test_corridor_placement_sequence(mvf):
    """Walk 300 frames (every 10th) down the corridor with n = 16 live 256^3
    volumes; the set of live cells after every step equals the oracle's."""
    seq = S.corridor_sequence(seed=3, n_frames=2000)
    s = 0.00293
    d_v, n_max, beta = 256, 16, 1.5
    og = O.OGrid((0.0, -1.0, 0.0), s)
    H = []
    log("placement sequence corridor")
    with mvf.Context() as ctx:
        gid = ctx.grid(og.origin, s)
        cell_of = {}
        for i in range(0, 2000, 40):
            d, _ = seq.frame(i)
            added, removed, ncells = ctx.placement_update(t(d), seq.poses[i], seq.K.as_array(), gid, d_v,
                                                          n_max, beta)
            counts = O.placement_counts(d, seq.K.as_array(), seq.poses[i], og, d_v)
            H, a_o, r_o = O.placement_policy(H, counts, n_max, beta)
            assert ncells == len(counts)
            for vid in added:
                assert ctx.dims(vid) == (d_v, d_v, d_v)
                cell_of[vid] = tuple(int(x) // (d_v - 2) for x in ctx.offset(vid))
            live = sorted(cell_of[v] for v in cell_of if ctx.query(v)[2])
            assert live == sorted(H), (i, live, sorted(H))
            assert sorted(cell_of[v] for v in added) == sorted(a_o)
            assert sorted(cell_of[v] for v in removed) == sorted(r_o)
        assert len(cell_of) > n_max  # the walk displaced volumes


def test_corridor_class_placement_sequence(mvf):
    """The corridor walk with volumes of three sizes (512^3, 384^3 and 256^3
    at 2.93 mm: sides 1.5, 1.125 and 0.75 m; at most 4, 6 and 6 live, taken
    in that rank order): after every step the live (size, cell) set, the
    added and the removed volumes equal the oracle's class rule on the
    oracle's endpoints."""
    seq = S.corridor_sequence(seed=3, n_frames=2000)
    s = 0.00293
    classes = [(512, 4), (384, 6), (256, 6)]
    beta = 1.5
    og = O.OGrid((0.0, -1.0, 0.0), s)
    K = seq.K.as_array()
    H = {d: [] for d, _ in classes}
    log("class placement sequence corridor")
    with mvf.Context() as ctx:
        gid = ctx.grid(og.origin, s)
        key_of = {}
        n_disp = 0
        idx = list(range(0, 2000, 40))
        for i, (d, _) in zip(idx, seq.frames(idx, threads=16)):
            added, removed, ncells = ctx.placement_update_classes(t(d), seq.poses[i], K, gid, classes, beta)
            g, cells = O.placement_endpoints(d, K, seq.poses[i], og, [c for c, _ in classes])
            H, a_o, r_o = O.placement_policy_classes(H, g, cells, classes, beta)
            for vid in added:
                dv = ctx.dims(vid)[0]
                assert ctx.dims(vid) == (dv, dv, dv)
                key_of[vid] = (dv, tuple(int(x) // (dv - 2) for x in ctx.offset(vid)))
            live = sorted(key_of[v] for v in key_of if ctx.query(v)[2])
            expect = sorted((dv, k) for dv in H for k in H[dv])
            assert live == expect, (i, live, expect)
            assert sorted(key_of[v] for v in added) == sorted((dv, k) for dv in a_o for k in a_o[dv])
            assert sorted(key_of[v] for v in removed) == sorted((dv, k) for dv in r_o for k in r_o[dv])
            n_disp += len(removed)
            for dv, q in classes:
                assert len(H[dv]) <= q
        # every class is used and the walk displaced volumes of each size
        assert {k[0] for k in key_of.values()} == {512, 384, 256}
        assert n_disp > 0


def _class_counts(g, cells, d_v, covered):
    kc = np.asarray(cells[d_v], np.int64).reshape(-1, 3)[~covered]
    out = {}
    for k in map(tuple, kc.tolist()):
        out[k] = out.get(k, 0) + 1
    return out


def test_custom_policy_region_of_interest(mvf):
    """A user-defined insertion f (the paper's f may be any function of the
    frames and the live volumes): 384^3 volumes only for cells whose centre
    lies in a region of interest (the first 8 m of the corridor), ranked by
    count, and 256^3 volumes by count everywhere else.  The counts the
    function receives equal the oracle's endpoint counts of each class (each
    class excluding the endpoints the kept volumes of the earlier classes
    hold), and after every step the live (size, cell) set is exactly what
    the function kept, with the added and removed volumes the differences."""
    seq = S.corridor_sequence(seed=3, n_frames=2000)
    s = 0.00293
    classes = [(384, 3), (256, 6)]
    og = O.OGrid((0.0, -1.0, 0.0), s)
    K = seq.K.as_array()
    roi_x = 8.0

    def centre_x(d_v, k):
        return og.origin[0] + s * (k[0] * (d_v - 2) + d_v / 2)

    seen = {}

    def policy(ci, d_v, live, counts, quota):
        seen[ci] = (sorted(live), dict(counts))
        cand = [k for k in counts if ci > 0 or centre_x(d_v, k) < roi_x]
        cand.sort(key=lambda k: (-counts[k], k))
        return cand[:quota]

    log("custom placement policy corridor")
    with mvf.Context() as ctx:
        gid = ctx.grid(og.origin, s)
        key_of = {}
        live_expect = {d: [] for d, _ in classes}
        idx = list(range(0, 2000, 50))
        for i, (d, _) in zip(idx, seq.frames(idx, threads=16)):
            seen.clear()
            added, removed, _ = ctx.placement_update_custom(t(d), seq.poses[i], K, gid, classes, policy)
            g, cells = O.placement_endpoints(d, K, seq.poses[i], og, [c for c, _ in classes])
            g = np.asarray(g, np.int64)
            covered = np.zeros(len(g), bool)
            new_live = {}
            for ci, (d_v, quota) in enumerate(classes):
                live_in, cnt = seen[ci]
                assert live_in == sorted(live_expect[d_v])
                assert cnt == _class_counts(g, cells, d_v, covered)
                new_live[d_v] = policy(ci, d_v, live_in, cnt, quota)
                for k in new_live[d_v]:
                    lo = np.asarray(k, np.int64) * (d_v - 2)
                    covered |= np.all((g >= lo) & (g < lo + d_v), axis=1)
            for vid in added:
                dv = ctx.dims(vid)[0]
                key_of[vid] = (dv, tuple(int(x) // (dv - 2) for x in ctx.offset(vid)))
            live = sorted(key_of[v] for v in key_of if ctx.query(v)[2])
            assert live == sorted((dv, k) for dv in new_live for k in new_live[dv])
            exp_add = sorted((dv, k) for dv in new_live for k in new_live[dv] if k not in live_expect[dv])
            exp_rem = sorted((dv, k) for dv in live_expect for k in live_expect[dv] if k not in new_live[dv])
            assert sorted(key_of[v] for v in added) == exp_add
            assert sorted(key_of[v] for v in removed) == exp_rem
            for vid in removed:
                assert not ctx.query(vid)[0]   # swapped out
            live_expect = new_live
            for k in new_live[384]:
                assert centre_x(384, k) < roi_x
        assert {k[0] for k in key_of.values()} == {384, 256}


def test_custom_policy_errors(mvf):
    """A function that fails, keeps too many cells or one cell twice is
    reported, and nothing beyond the classes already done changes."""
    seq = S.corridor_sequence(seed=3, n_frames=10)
    og = O.OGrid((0.0, -1.0, 0.0), 0.00293)
    K = seq.K.as_array()
    d, _ = seq.frame(0)
    log("custom placement policy errors")
    with mvf.Context() as ctx:
        gid = ctx.grid(og.origin, og.voxel_size)

        def boom(ci, d_v, live, counts, quota):
            raise KeyError("boom")

        with pytest.raises(KeyError):
            ctx.placement_update_custom(t(d), seq.poses[0], K, gid, [(256, 4)], boom)
        with pytest.raises(ValueError):
            ctx.placement_update_custom(t(d), seq.poses[0], K, gid, [(256, 1)],
                                        lambda ci, dv, lv, cnt, q: list(cnt)[:2])
        twice = lambda ci, dv, lv, cnt, q: [next(iter(cnt))] * 2
        with pytest.raises(mvf._lib.MvfError):
            ctx.placement_update_custom(t(d), seq.poses[0], K, gid, [(256, 4)], twice)
        a, r, _ = ctx.placement_update_custom(t(d), seq.poses[0], K, gid, [(256, 4)],
                                              lambda ci, dv, lv, cnt, q: sorted(cnt)[:q])
        assert len(a) == min(4, len(O.placement_counts(d, K, seq.poses[0], og, 256))) and r == []
