"""Pins for the oracle's placement step (Dynamic Mapping for SLAM and
Insertion and Removal sections of the paper)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from synth import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "placement_policy_cases.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_policy_golden(case):
    counts = {tuple(k): c for k, c in case["counts"]}
    H, added, removed = O.placement_policy([tuple(a) for a in case["active"]], counts,
                                           case["n"], case["beta"])
    assert sorted(H) == sorted(tuple(a) for a in case["expect_active"])
    assert sorted(added) == sorted(tuple(a) for a in case["expect_added"])
    assert sorted(removed) == sorted(tuple(a) for a in case["expect_removed"])
    assert len(H) <= case["n"] and len(set(H)) == len(H)


def test_counts_fronto_parallel_plane():
    """Camera at the origin looking down +z at a plane 1.5 m away; the cell
    of side L = s (d_v - 2) = 1 m containing each endpoint is known from the
    pixel column/row alone, so the counts follow from integer pixel
    intervals: along x the cell boundaries e_x = -0.3 and 0.7 fall between
    columns 29|30 and 96|97."""
    w, h = 100, 80
    K = np.array([100.0, 100.0, 49.5, 39.5], np.float32)
    T = np.zeros((3, 4))
    T[:, :3] = np.eye(3)
    grid = O.OGrid((-2.3, -2.0, -2.0), 1.0 / 64)
    depth = np.full((h, w), 1.5, np.float32)
    depth[0, 0] = 0.0
    depth[5, 7] = np.nan
    c = O.placement_counts(depth, K, T, grid, d_v=66)
    # x: e_x = 1.5 (u - 49.5) / 100; cells floor((e_x + 2.3) / 1)
    ux = {1: range(0, 30), 2: range(30, 97), 3: range(97, 100)}
    # y: e_y = 1.5 (v - 39.5) / 100 in [-0.5925, 0.5925]; +2 -> cells 1 and 2 split at v = 40
    vy = {1: range(0, 40), 2: range(40, 80)}
    expect = {}
    for kx, us in ux.items():
        for ky, vs in vy.items():
            n = len(us) * len(vs)
            n -= sum(1 for (vv, uu) in [(0, 0), (5, 7)] if uu in us and vv in vs)
            expect[(kx, ky, 3)] = n
    assert c == expect
    assert sum(c.values()) == w * h - 2


def test_endpoints_fall_in_their_cells():
    """For a real frame every counted ray endpoint, recomputed in binary64
    from depth, intrinsics and pose, lies inside (up to rounding) the cell
    it was counted in."""
    seq = S.small_room_sequence()
    d, _ = seq.frame(2)
    T = seq.poses[2]
    K = seq.K.as_array()
    grid = O.OGrid((-2.0, -2.0, -2.0), 4.0 / 256)
    d_v = 66
    L = grid.voxel_size * (d_v - 2)
    h, w = d.shape
    cells = np.zeros((h * w, 3), np.int32)
    valid = np.zeros(h * w, np.uint8)
    O.lib().orc_placement_cells(O._p(d), w, h, O._p(K), O._p(np.asarray(T, np.float32).reshape(12)),
                                O._p(grid.arr4()), d_v, O._p(cells), O._p(valid))
    u, v = np.meshgrid(np.arange(w), np.arange(h))
    q = np.stack([d * (u - K[2]) / K[0], d * (v - K[3]) / K[1], d], -1).reshape(-1, 3)
    e = q @ np.asarray(T, np.float32).astype(np.float64)[:, :3].T + np.asarray(T, np.float32)[:, 3]
    rel = (e - np.asarray(grid.origin)) / L - cells
    assert valid.all()
    assert rel.min() > -1e-5 and rel.max() < 1 + 1e-5
    counts = O.placement_counts(d, K, T, grid, d_v)
    assert sum(counts.values()) == w * h and len(counts) >= 4


# -- volumes of several sizes (Dynamic Mapping for SLAM: f chooses the
# volume parameters, here the size by count rank) --------------------------

CLASS_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "placement_class_cases.json")


def _class_cases():
    with open(CLASS_GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _class_cases(), ids=lambda c: c["name"])
def test_class_policy_golden(case):
    g, cells = [], {d: [] for d, _ in case["classes"]}
    for gx, n in case["endpoints"]:
        for _ in range(n):
            g.append((gx, 0, 0))
            for d in cells:
                cells[d].append((gx // (d - 2), 0, 0))
    active = {int(d): [tuple(k) for k in v] for d, v in case["active"].items()}
    H, added, removed = O.placement_policy_classes(active, np.array(g).reshape(-1, 3),
                                                   {d: np.array(v).reshape(-1, 3) for d, v in cells.items()},
                                                   [tuple(c) for c in case["classes"]], case["beta"])
    for d, quota in case["classes"]:
        key = str(d)
        assert sorted(H[d]) == sorted(tuple(k) for k in case["expect_active"][key]), (d, H[d])
        assert sorted(added[d]) == sorted(tuple(k) for k in case["expect_added"][key]), (d, added[d])
        assert sorted(removed[d]) == sorted(tuple(k) for k in case["expect_removed"][key]), (d, removed[d])
        assert len(H[d]) <= quota and len(set(H[d])) == len(H[d])


def test_one_class_is_the_single_size_rule():
    """With one class nothing is excluded: the step equals the single-size
    rule on the same frame's counts."""
    seq = S.small_room_sequence()
    K = seq.K.as_array()
    grid = O.OGrid((-2.0, -2.0, -2.0), 4.0 / 256)
    d_v = 34
    active = []
    for i in range(6):
        d, _ = seq.frame(i)
        counts = O.placement_counts(d, K, seq.poses[i], grid, d_v)
        H1, a1, r1 = O.placement_policy(active, counts, 5, 1.5)
        g, cells = O.placement_endpoints(d, K, seq.poses[i], grid, [d_v])
        H2, a2, r2 = O.placement_policy_classes({d_v: active}, g, cells, [(d_v, 5)], 1.5)
        assert (H1, a1, r1) == (H2[d_v], a2[d_v], r2[d_v])
        active = H1


def test_endpoint_voxels_match_binary64_geometry():
    """The voxel g each counted endpoint is assigned to (the side-one
    lattice) contains the endpoint recomputed in binary64, up to rounding
    at the faces, and the class cell of an endpoint equals floor(g / (d_v -
    2)) except for endpoints that rounding puts on the other side of a cell
    face (a sliver of at most a few ulp)."""
    seq = S.small_room_sequence()
    d, _ = seq.frame(4)
    T = seq.poses[4]
    K = seq.K.as_array()
    grid = O.OGrid((-2.0, -2.0, -2.0), 4.0 / 256)
    g, cells = O.placement_endpoints(d, K, T, grid, [34, 66])
    h, w = d.shape
    u, v = np.meshgrid(np.arange(w), np.arange(h))
    ok = (d > 0) & np.isfinite(d)
    q = np.stack([d * (u - K[2]) / K[0], d * (v - K[3]) / K[1], d], -1)[ok].astype(np.float64)
    T32 = np.asarray(T, np.float32).astype(np.float64)
    e = q @ T32[:, :3].T + T32[:, 3]
    rel = (e - np.asarray(grid.arr4()[:3], np.float64)) / np.float64(np.float32(grid.voxel_size)) - g
    assert len(g) == ok.sum()
    assert rel.min() > -1e-3 and rel.max() < 1 + 1e-3
    for dv, kc in cells.items():
        same = np.all(np.floor_divide(g, dv - 2) == kc, axis=1)
        assert same.mean() > 0.999, (dv, same.mean())
