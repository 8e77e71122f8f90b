"""Pins for the oracle's depth gradient (the differentiable raycast: pose
and voxel derivatives of the raycast depth with the discrete structure of
the march -- crossing index and sample cells -- held fixed).

The analytic binary64 gradient is checked against binary64 central finite
differences of the binary64 forward, and on a linear field against the
derivative of the analytic ray-plane depth."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S


def _fused_volume(n=64):
    seq = S.small_room_sequence(noise=False)
    grid = O.OGrid((-1.0, -1.0, -1.0), 2.0 / n, 4.0, 128)
    vol = O.OVolume.empty((n, n, n))
    K = seq.K.as_array()
    for i in range(10):
        d, rgb = seq.frame(i)
        O.integrate(vol, grid, d, rgb, K, seq.poses[i])
    return seq, grid, vol, K


@pytest.fixture(scope="module")
def fused():
    return _fused_volume()


def _pose_fd(vol, grid, K, T, w, h, kc, gd, eps=1e-6):
    out = np.zeros(6)
    for i in range(6):
        e = np.zeros(6)
        e[i] = eps
        zp = O.depth_fixed(vol, grid, K, O.compose(T, O.se3_exp(e)), w, h, kc)
        zm = O.depth_fixed(vol, grid, K, O.compose(T, O.se3_exp(-e)), w, h, kc)
        out[i] = np.sum(gd * (zp - zm)) / (2 * eps)
    return out


def test_pose_gradient_matches_central_differences(fused):
    seq, grid, vol, K = fused
    T = S.perturb_pose(seq.poses[4], np.random.default_rng(5), 0.02, 2.0)
    T32 = np.asarray(T, np.float32).astype(np.float64)
    w, h = 320, 240
    rc = O.raycast([vol], grid, K, T32, w, h)
    kc = O.structure(rc)
    assert (kc[:, 0] >= 0).mean() > 0.2
    # ill-conditioned crossings (F_a - F_b < 1e-3, flagged ambiguous) have huge
    # third derivatives that swamp the O(h^2) finite-difference error
    ok = (rc["hit"] >= 0) & (rc["ambiguous"] == 0)
    gd = np.random.default_rng(1).normal(size=(h, w)) * ok
    g, _ = O.depth_grad(vol, grid, K, T32, w, h, kc, gd, want_voxels=False)
    fd = _pose_fd(vol, grid, K, T32, w, h, kc, gd)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())


def test_voxel_gradient_matches_central_differences(fused):
    seq, grid, vol, K = fused
    T = np.asarray(seq.poses[7], np.float32).astype(np.float64)
    w, h = 160, 120
    Ks = np.array([K[0] / 2, K[1] / 2, (K[2] - 0.5) / 2, (K[3] - 0.5) / 2], np.float32)
    rc = O.raycast([vol], grid, Ks, T, w, h)
    kc = O.structure(rc)
    gd = np.random.default_rng(2).normal(size=(h, w)) * ((rc["hit"] >= 0) & (rc["ambiguous"] == 0))
    _, gF = O.depth_grad(vol, grid, Ks, T, w, h, kc, gd)
    F32 = vol.F32()
    idx = np.argwhere(np.abs(gF) > 1e-3 * np.abs(gF).max())
    assert len(idx) > 100
    rng = np.random.default_rng(3)
    for j in rng.choice(len(idx), 25, replace=False):
        z, y, x = idx[j]
        Fp, Fm = F32.copy(), F32.copy()
        Fp[z, y, x] += np.float32(1e-3)
        Fm[z, y, x] -= np.float32(1e-3)
        dp = O.depth_fixed(vol, grid, Ks, T, w, h, kc, F32=Fp)
        dm = O.depth_fixed(vol, grid, Ks, T, w, h, kc, F32=Fm)
        step = float(Fp[z, y, x]) - float(Fm[z, y, x])
        fd = np.sum(gd * (dp - dm)) / step
        assert abs(fd - gF[z, y, x]) <= 1e-4 * abs(gF[z, y, x]) + 1e-12, (fd, gF[z, y, x])
    # voxels no crossing touches get no gradient
    touched = np.zeros(vol.W.shape, bool)
    kcr = kc[kc[:, 0] >= 0]
    for cell in (kcr[:, 1:4], kcr[:, 4:7]):
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    touched[cell[:, 2] + dz, cell[:, 1] + dy, cell[:, 0] + dx] = True
    assert np.all(gF[~touched] == 0)


def test_linear_field_pose_gradient_closed_form():
    """On a linear field the fixed-structure depth is the analytic ray-plane
    depth z(T) = dz_c (d0 - n.C) / (n.R dz), whose pose derivative is taken
    here by finite differences of that closed form."""
    grid = O.OGrid((-1.0, -1.0, -1.0), 1.0 / 32, 4.0)
    vol = O.OVolume.empty((64, 64, 64))
    rng = np.random.default_rng(9)
    n = np.array([0.2, -0.3, 1.0])
    n /= np.linalg.norm(n)
    d0 = 0.05
    s = grid.voxel_size
    nz_, ny_, nx_ = vol.W.shape
    gz, gy, gx = np.meshgrid(np.arange(nz_), np.arange(ny_), np.arange(nx_), indexing="ij")
    x = np.stack([-1 + s * (gx + 0.5), -1 + s * (gy + 0.5), -1 + s * (gz + 0.5)], -1)
    vol.F[:] = (x @ n - d0) / grid.mu
    vol.W[:] = 1
    T = S.look_at(n * 0.9 + np.array([0.1, 0.05, 0.0]), [0.0, 0.0, 0.0], up=(0, 1, 0))
    T = np.asarray(T, np.float32).astype(np.float64)
    K = np.array([80.0, 80.0, 31.5, 23.5], np.float32)
    w, h = 64, 48
    rc = O.raycast([vol], grid, K, T, w, h)
    kc = O.structure(rc)
    hit = rc["hit"] >= 0
    assert hit.mean() > 0.9
    gd = rng.normal(size=(h, w)) * hit

    u, v = np.meshgrid(np.arange(w, dtype=np.float64), np.arange(h, dtype=np.float64))
    dc = np.stack([(u - K[2]) / K[0], (v - K[3]) / K[1], np.ones_like(u)], -1)
    dh = dc / np.linalg.norm(dc, axis=-1, keepdims=True)

    def z_analytic(Tp):
        dw = dh @ Tp[:, :3].T
        t = (d0 - Tp[:, 3] @ n) / (dw @ n)
        return t * dh[..., 2]

    np.testing.assert_allclose(O.depth_fixed(vol, grid, K, T, w, h, kc)[hit], z_analytic(T)[hit],
                               atol=1e-6)
    g, _ = O.depth_grad(vol, grid, K, T, w, h, kc, gd, want_voxels=False)
    ref = np.zeros(6)
    for i in range(6):
        e = np.zeros(6)
        e[i] = 1e-6
        ref[i] = np.sum(gd * (z_analytic(O.compose(T, O.se3_exp(e)))
                              - z_analytic(O.compose(T, O.se3_exp(-e))))) / 2e-6
    np.testing.assert_allclose(g, ref, rtol=2e-5, atol=1e-7 * np.abs(ref).max())
