"""Pins of the oracle's camera tracking (Depth Map Conversion; Camera
Tracking: projective point-to-plane ICP).

- vertex and normal maps of planes: a fronto-parallel plane gives vertices
  at its depth and the normal (0, 0, 1) exactly; a tilted plane gives
  normals parallel to its own normal; missing neighbours give none;
- the depth pyramid: constant maps stay constant, outliers beyond tau leave
  the block mean, empty blocks give 0, hand-computed blocks;
- the normal equations: b is half the gradient and A half the Hessian of
  the point-to-plane energy E(xi) = sum (n_m . (Exp(xi) v_g - v_m))^2 with
  the associations held (central differences in binary64, at a zero-residual
  configuration where the Gauss-Newton Hessian is exact);
- tracking: a frame tracked against the maps of its own pose stays put; a
  frame rendered at a pose 2 cm / 1.5 degrees away from the model's is
  tracked back to its true pose.
"""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S

K = np.array([525.0, 525.0, 319.5, 239.5], np.float32)


def test_fronto_parallel_plane_exact():
    d = np.full((480, 640), 2.5, np.float32)
    V, N = O.vertex_normal(d, K)
    assert np.all(V[..., 2] == np.float32(2.5))
    ok = np.isfinite(N).all(axis=2)
    assert ok[:-1, :-1].all() and not ok[-1].any() and not ok[:, -1].any()
    assert np.all(N[:-1, :-1] == np.array([0, 0, 1], np.float32))
    # x of a vertex: (x - cx) / fx * d, its sign and size by integer geometry
    assert V[0, 0, 0] < 0 < V[0, 639, 0] and V[0, 0, 1] < 0 < V[479, 0, 1]
    assert abs(V[10, 20, 0] - (20 - 319.5) / 525.0 * 2.5) < 1e-6


def test_tilted_plane_normals_parallel():
    # plane n . p = 3 with a tilted unit normal, seen from the origin
    n = np.array([0.3, -0.2, 1.0])
    n /= np.linalg.norm(n)
    h, w = 60, 80
    u, v = np.meshgrid(np.arange(w), np.arange(h))
    ray = np.stack([(u - K[2]) / K[0], (v - K[3]) / K[1], np.ones_like(u, float)], -1)
    z = 3.0 / (ray @ n)                    # z-depth: p = ray * z
    V, N = O.vertex_normal(z.astype(np.float32), K)
    ok = np.isfinite(N).all(axis=2)
    assert ok.sum() == (h - 1) * (w - 1)
    cos = np.abs(N[ok].astype(np.float64) @ n)
    assert cos.min() > 1 - 1e-6
    # points lie on the plane
    assert np.abs(V.reshape(-1, 3).astype(np.float64) @ n - 3.0).max() < 1e-5


def test_missing_neighbours_give_no_normal():
    d = np.full((10, 10), 1.0, np.float32)
    d[4, 5] = 0.0
    d[7, 2] = np.nan
    d[2, 8] = np.inf
    V, N = O.vertex_normal(d, K)
    bad = ~np.isfinite(N).all(axis=2)
    for (y, x) in [(4, 5), (7, 2), (2, 8)]:
        assert np.isnan(V[y, x]).all()
        assert bad[y, x] and bad[y, x - 1] and bad[y - 1, x]   # the pixel and those that use it
    assert not bad[0, 0]


def test_depth_pyramid_blocks():
    assert np.all(O.depth_pyramid(np.full((8, 12), 1.7, np.float32), 3)[2] == np.float32(1.7))
    d = np.zeros((4, 4), np.float32)
    d[0:2, 0:2] = [[1.0, 1.02], [1.5, 0.99]]      # 1.5 is an outlier to the block's first depth
    d[0:2, 2:4] = [[0.0, 2.0], [2.01, np.nan]]    # first valid is 2.0
    d[2:4, 0:2] = 0.0                             # empty
    d[2:4, 2:4] = [[3.0, 3.0], [3.0, 3.03]]       # 3.03 - 3.0 rounds above 0.03
    d2 = O.depth_pyramid(d, 2)[1]
    assert d2.shape == (2, 2)
    assert d2[0, 0] == np.float32((np.float32(1.0) + np.float32(1.02)) + np.float32(0.99)) / np.float32(3)
    assert d2[0, 1] == np.float32(np.float32(2.0) + np.float32(2.01)) / np.float32(2)
    assert d2[1, 0] == 0.0
    keep = np.float32(np.float32(3.03) - np.float32(3.0)) <= np.float32(0.03)
    exp = (np.float32(12.03) / 4) if keep else np.float32(9.0) / 3
    assert abs(d2[1, 1] - exp) < 1e-6
    # odd sizes: the last row / column is dropped
    assert O.depth_pyramid(np.ones((7, 9), np.float32), 2)[1].shape == (3, 4)


def test_level_intrinsics():
    K1 = O.level_K(K, 1)
    assert list(K1) == [262.5, 262.5, 159.5, 119.5]
    # pixel centres map onto the level's centres: x_l = (x_0 + 1/2) / 2 - 1/2
    K2 = O.level_K(K, 2)
    assert K2[2] == np.float32((319.5 + 0.5) / 4 - 0.5)


def _room_frame(T, K_=K, w=640, h=480, noise=False):
    seq = S.large_room_sequence(seed=2, n_frames=2, noise=False)
    Kin = S.Intrinsics(float(K_[0]), float(K_[1]), float(K_[2]), float(K_[3]), w, h)
    d, _, _ = S.render(seq.scene, Kin, T)
    return seq, d


def _model_maps(depth, T):
    """World vertex and normal maps of a depth frame at pose T (the model a
    raycast of a perfect map would give)."""
    V, N = O.vertex_normal(depth, K)
    R, t = np.asarray(T, np.float64)[:, :3], np.asarray(T, np.float64)[:, 3]
    Vw = (V.reshape(-1, 3).astype(np.float64) @ R.T + t).astype(np.float32).reshape(V.shape)
    Nw = (N.reshape(-1, 3).astype(np.float64) @ R.T).astype(np.float32).reshape(N.shape)
    return Vw, Nw


def _moved_vertices(V, T):
    """v_g = R v + t of the oracle's association, replayed with binary32
    numpy operations in the same order (one rounding each)."""
    T32 = np.asarray(T, np.float32)
    v = V.astype(np.float32)
    out = np.empty_like(v)
    for a in range(3):
        out[:, a] = (((T32[a, 0] * v[:, 0]) + (T32[a, 1] * v[:, 1])) + (T32[a, 2] * v[:, 2])) + T32[a, 3]
    return out.astype(np.float64)


@pytest.mark.parametrize("offset_mm", [0.0, 8.0])
def test_normal_equations_are_the_energy_derivatives(offset_mm):
    """With the associations held, b is half the gradient of the
    point-to-plane energy at xi = 0; at zero residual (the estimate equals
    the model's pose) A is half its Hessian."""
    seq = S.large_room_sequence(seed=2, n_frames=3, noise=False)
    Tm = seq.poses[1]
    Kin = S.Intrinsics(262.5, 262.5, 159.5, 119.5, 320, 240)
    Kq = Kin.as_array()
    d, _, _ = S.render(seq.scene, Kin, Tm)
    V, N = O.vertex_normal(d, Kq)
    R, t = Tm[:, :3], Tm[:, 3]
    Vm = (V.reshape(-1, 3).astype(np.float64) @ R.T + t).astype(np.float32).reshape(V.shape)
    Nm = (N.reshape(-1, 3).astype(np.float64) @ R.T).astype(np.float32).reshape(N.shape)
    T = Tm.copy()
    T[:, 3] += np.array([0.6, -0.3, 0.74]) * offset_mm * 1e-3
    A, b, n, e, inl = O.icp_reduce(V, N, Vm, Nm, Kq, T, Tm)
    assert n > 0.5 * np.isfinite(N).all(axis=2).sum()
    m = inl.astype(bool)
    vg = _moved_vertices(V[m], T)
    # the model pixel each inlier was paired with, by the same projection
    Tm32 = np.asarray(Tm, np.float32)
    dd = (vg.astype(np.float32) - Tm32[:, 3]).astype(np.float32)
    q = np.stack([((Tm32[0, a] * dd[:, 0]) + (Tm32[1, a] * dd[:, 1])) + (Tm32[2, a] * dd[:, 2]) for a in range(3)], 1)
    iz = (np.float32(1.0) / q[:, 2]).astype(np.float32)
    ur = np.floor((((Kq[0] * q[:, 0]) * iz) + Kq[2]) + np.float32(0.5)).astype(np.int64)
    vr = np.floor((((Kq[1] * q[:, 1]) * iz) + Kq[3]) + np.float32(0.5)).astype(np.int64)
    vm = Vm[vr, ur].astype(np.float64)
    nm = Nm[vr, ur].astype(np.float64)

    def E(xi):
        X = O.se3_exp(xi)
        p = vg @ X[:, :3].T + X[:, 3]
        r = np.einsum("ij,ij->i", nm, p - vm)
        return float(r @ r)

    assert abs(E(np.zeros(6)) - e) <= 1e-9 * max(e, 1e-30) + 1e-18
    if offset_mm > 0.0:
        # (at zero offset b holds only rounding residuals, below what a
        # difference quotient resolves)
        h = 1e-6
        grad = np.array([(E(h * np.eye(6)[i]) - E(-h * np.eye(6)[i])) / (2 * h) for i in range(6)])
        assert np.abs(b - 0.5 * grad).max() <= 1e-7 * np.abs(b).max()
    else:
        hh = 1e-4
        H = np.zeros((6, 6))
        for i in range(6):
            for j in range(6):
                ei, ej = hh * np.eye(6)[i], hh * np.eye(6)[j]
                H[i, j] = (E(ei + ej) - E(ei - ej) - E(-ei + ej) + E(-ei - ej)) / (4 * hh * hh)
        assert np.allclose(A, 0.5 * H, rtol=1e-3, atol=1e-3 * np.abs(H).max())


def test_tracking_stays_put_on_its_own_maps():
    seq = S.large_room_sequence(seed=2, n_frames=3, noise=False)
    T = seq.poses[1]
    d, _, _ = S.render(seq.scene, seq.K, T)
    Vm, Nm = _model_maps(d, T)
    T1, log = O.icp_track(d, K, Vm, Nm, T, T, smooth=0.0)
    assert np.abs(T1 - T).max() < 1e-5
    # smoothed, against maps of the same smoothed depth
    ds = O.depth_smooth(d)
    Vs, Ns = _model_maps(ds, T)
    T1, log = O.icp_track(d, K, Vs, Ns, T, T)
    assert np.abs(T1 - T).max() < 1e-5
    assert log[-1][1] > 100000


@pytest.mark.parametrize("seed", [0, 1])
def test_tracking_recovers_a_known_motion(seed):
    """Model maps from the frame at pose T0; the frame at T1 = T0 Exp(delta)
    (2 cm, 1.5 degrees) is tracked from T0 back to T1."""
    seq = S.large_room_sequence(seed=2, n_frames=60, noise=False)
    T0 = seq.poses[10 + 20 * seed]
    rng = np.random.default_rng(40 + seed)
    T1 = S.perturb_pose(T0, rng, 0.02, 1.5)
    d0, _, _ = S.render(seq.scene, seq.K, T0)
    d1, _, _ = S.render(seq.scene, seq.K, T1)
    Vm, Nm = _model_maps(d0, T0)
    T, log = O.icp_track(d1, K, Vm, Nm, T0, T0, smooth=0.0)
    et = np.linalg.norm(T[:, 3] - T1[:, 3])
    R = T[:, :3].T @ T1[:, :3]
    er = np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    assert et < 1e-3 and er < 0.05, (et, er)
    # and the error decreased along the way
    assert log[-1][2] / max(1, log[-1][1]) < log[0][2] / max(1, log[0][1])


def test_smoothing_constant_step_hole_and_noise():
    """Edge-preserving smoothing: a two-level step (levels 1 m and 2 m, more
    than delta apart) keeps each side's value exactly (integer weights and
    exactly representable depths); a hole neither spreads nor is filled; a
    ramp is reproduced inside the image (a symmetric window of a linear
    function); i.i.d. noise on a plane shrinks by the kernel's factor
    sqrt(sum of the squared normalised weights) = 924 / 4096."""
    d = np.ones((40, 50), np.float32)
    d[:, 25:] = 2.0
    d[10, 10] = 0.0
    d[30, 40] = np.nan
    s = O.depth_smooth(d, 0.09)
    ok = np.isfinite(d) & (d > 0)
    assert np.array_equal(s[ok], d[ok])
    assert s[10, 10] == 0.0 and s[30, 40] == 0.0
    # ramp along x: exact in the interior up to rounding
    x = np.arange(60, dtype=np.float32)
    ramp = np.tile(np.float32(1.5) + np.float32(0.001) * x, (30, 1)).astype(np.float32)
    sr = O.depth_smooth(ramp, 0.09)
    assert np.abs(sr[3:-3, 3:-3] - ramp[3:-3, 3:-3]).max() < 2e-6
    # noise
    rng = np.random.default_rng(3)
    noisy = (2.0 + rng.normal(0, 0.005, (200, 200))).astype(np.float32)
    sn = O.depth_smooth(noisy, 0.09)[10:-10, 10:-10]
    ratio = float((sn - 2.0).std() / (noisy[10:-10, 10:-10] - 2.0).std())
    assert abs(ratio - 924 / 4096) < 0.02, ratio


def test_tracking_noisy_frames_with_smoothing():
    """With depth noise (sigma 1.5 mm z^2) the smoothed frames still track a
    known 2 cm / 1.5 degree motion back to within 3 mm / 0.2 degree."""
    seq = S.large_room_sequence(seed=2, n_frames=60, noise=True)
    T0 = seq.poses[20]
    T1 = S.perturb_pose(T0, np.random.default_rng(44), 0.02, 1.5)
    d0, _, _ = S.render(seq.scene, seq.K, T0)      # model: noise-free
    d1, _, _ = S.render(seq.scene, seq.K, T1)
    d1 = S.add_depth_noise(d1, 2, 21)
    Vm, Nm = _model_maps(d0, T0)
    T, log = O.icp_track(d1, K, Vm, Nm, T0, T0)
    et = np.linalg.norm(T[:, 3] - T1[:, 3])
    R = T[:, :3].T @ T1[:, :3]
    er = np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))
    assert et < 3e-3 and er < 0.2, (et, er)
