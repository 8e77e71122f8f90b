"""Differentiable raycast on the device vs the oracle: forward depth and
crossing record, backward pose and voxel gradients vs the binary64 CPU
gradient, and pose refinement by gradient descent."""
import numpy as np
import pytest

import oracle as O
from synth import scenes as S
from tests.util import dev, log, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mvf():
    import paper_1511_07106_amd as mvf
    return mvf


@pytest.fixture(scope="module")
def fused():
    seq = S.small_room_sequence(seed=1, noise=False)
    n = 96
    og = O.OGrid((-1.0, -1.0, -1.0), 2.0 / n, 4.0, 128)
    ov = O.OVolume.empty((n, n, n))
    K = seq.K.as_array()
    for i in range(10):
        d, c = seq.frame(i)
        O.integrate(ov, og, d, c, K, seq.poses[i])
    return seq, og, ov


def _dense(ov):
    import torch
    F = t(ov.F32())
    W = torch.from_numpy(ov.W.view(np.int16).copy()).to(dev())
    return F, W


def test_forward_matches_oracle(mvf, fused):
    seq, og, ov = fused
    K = seq.K.as_array()
    T = S.perturb_pose(seq.poses[4], np.random.default_rng(3), 0.02, 2.0)
    log("diffray forward 96^3")
    with mvf.Context() as ctx:
        F, W = _dense(ov)
        depth, record = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T, K, 320, 240)
        rc = O.raycast([ov], og, K, T, 320, 240)
        rec = record.cpu().numpy()
        np.testing.assert_array_equal(rec, rc["k"])
        hit = rec >= 0
        assert hit.mean() > 0.2
        dd = np.abs(depth.cpu().numpy().astype(np.float64) - rc["depth"])[hit]
        assert dd.max() <= 1e-4


def test_forward_generation_reuses_and_rebuilds(mvf, fused):
    """The forward's copy of (F, W): a non-zero generation reuses it (the
    same results as a rebuild on every call), a new generation after F
    changed rebuilds it (the result follows the new field), and a second
    volume of another shape replaces it."""
    import torch
    seq, og, ov = fused
    K = seq.K.as_array()
    T = S.perturb_pose(seq.poses[2], np.random.default_rng(13), 0.02, 2.0)
    log("diffray forward generations 96^3")
    with mvf.Context() as ctx:
        F, W = _dense(ov)
        d0, r0 = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T, K, 320, 240)
        d1, r1 = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T, K, 320, 240, generation=7)
        d2, r2 = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T, K, 320, 240, generation=7)
        assert torch.equal(d0, d1) and torch.equal(d1, d2) and torch.equal(r0, r2)
        # shift the field by a quarter voxel's worth of truncation units
        F2 = F - 0.0625
        F.copy_(F2)
        F32 = (ov.F32() - np.float32(0.0625)).astype(np.float32)
        d3, r3 = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T, K, 320, 240, generation=8)
        rc = O.raycast([ov], og, K, T, 320, 240, F32=[F32])
        np.testing.assert_array_equal(r3.cpu().numpy(), rc["k"])
        hit = rc["k"] >= 0
        dd = np.abs(d3.cpu().numpy().astype(np.float64) - rc["depth"])[hit]
        assert dd.max() <= 1e-4
        assert not torch.equal(d3, d1)
        # another shape: a crop of the volume
        Fc, Wc = F[8:72, 4:90, 10:60].contiguous(), W[8:72, 4:90, 10:60].contiguous()
        d4, r4 = ctx.diffray_forward(Fc, Wc, og.origin, og.voxel_size, T, K, 320, 240, offset=(10, 4, 8),
                                     generation=8)
        crop = O.OVolume((50, 86, 64), (10, 4, 8), F32[8:72, 4:90, 10:60].astype(np.float64),
                         ov.W[8:72, 4:90, 10:60].copy(), np.zeros((64, 86, 50, 4), np.uint8))
        rc4 = O.raycast([crop], og, K, T, 320, 240, F32=[F32[8:72, 4:90, 10:60].copy()])
        np.testing.assert_array_equal(r4.cpu().numpy(), rc4["k"])


def test_backward_matches_oracle_gradient(mvf, fused):
    seq, og, ov = fused
    K = seq.K.as_array()
    T = S.perturb_pose(seq.poses[6], np.random.default_rng(4), 0.02, 2.0)
    T32 = np.asarray(T, np.float32).astype(np.float64)
    w, h = 320, 240
    log("diffray backward 96^3")
    import torch
    with mvf.Context() as ctx:
        F, W = _dense(ov)
        depth, record = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T32, K, w, h)
        rc = O.raycast([ov], og, K, T32, w, h)
        kc = O.structure(rc)
        gd = np.random.default_rng(5).normal(size=(h, w)).astype(np.float32) * (rc["hit"] >= 0)
        grad_F = torch.zeros_like(F)
        gxi = ctx.diffray_backward(F, W, og.origin, og.voxel_size, T32, K, t(gd), record, grad_F)
        g_ref, gF_ref = O.depth_grad(ov, og, K, T32, w, h, kc, gd.astype(np.float64))
        g = gxi.cpu().numpy()
        rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
        assert rel <= 1e-3, (g, g_ref)
        gF = grad_F.cpu().numpy().astype(np.float64)
        err = np.abs(gF - gF_ref).max() / np.abs(gF_ref).max()
        assert err <= 1e-3, err


def test_autograd_function_and_descent(mvf, fused):
    """The autograd.Function gives the same gradient as the direct call, and
    gradient descent on the pose reduces the depth residual and pose error."""
    import torch
    from paper_1511_07106_amd.autograd import DiffRaycast, depth_loss
    seq, og, ov = fused
    K = seq.K.as_array()
    w, h = 320, 240
    T_true = seq.poses[3]
    target_np = S.render(seq.scene, seq.K, T_true)[0]
    log("diffray autograd + 30 GD steps")
    with mvf.Context() as ctx:
        F, W = _dense(ov)
        target = t(target_np)
        T0 = S.perturb_pose(T_true, np.random.default_rng(11), 0.02, 2.0)
        err0 = np.linalg.norm(T0[:, 3] - T_true[:, 3])
        losses = []
        for it in range(30):
            xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
            Fg = F.clone().requires_grad_(True)
            depth = DiffRaycast.apply(Fg, xi, W, ctx, og.origin, og.voxel_size, T0, K, w, h)
            loss = depth_loss(depth, target)
            loss.backward()
            losses.append(float(loss))
            g = xi.grad.numpy()
            if it == 0:
                assert Fg.grad is not None and torch.isfinite(Fg.grad).all()
            step = 0.5 * g
            T0 = mvf.pose_retract(T0, -step)
        err1 = np.linalg.norm(T0[:, 3] - T_true[:, 3])
        assert losses[-1] < 0.2 * losses[0], losses
        assert err1 < err0


def test_autograd_gradient_at_nonzero_xi(mvf, fused):
    """Through the autograd.Function at xi != 0: dL/dxi equals binary64
    central differences in xi of the oracle's fixed-structure depth at
    T0 Exp(xi +- h e_i) (so xi can be kept as a parameter and stepped)."""
    import torch
    from paper_1511_07106_amd.autograd import DiffRaycast
    seq, og, ov = fused
    K = seq.K.as_array()
    w, h = 320, 240
    T0 = seq.poses[2]
    xi0 = np.array([0.02, -0.015, 0.01, 0.03, -0.04, 0.02])
    gd = np.random.default_rng(8).normal(size=(h, w))
    log("diffray autograd at nonzero xi 96^3")
    with mvf.Context() as ctx:
        F, W = _dense(ov)
        xi = torch.tensor(xi0, dtype=torch.float64, requires_grad=True)
        depth = DiffRaycast.apply(F, xi, W, ctx, og.origin, og.voxel_size, T0, K, w, h)
        hit = (depth > 0).cpu().numpy()
        gdm = gd * hit
        loss = (depth.double() * t(gdm)).sum()
        loss.backward()
        g = xi.grad.numpy()
        # the structure the forward froze, from the oracle at the same binary32 pose
        T = mvf.pose_retract(T0, xi0)
        T32 = np.asarray(T, np.float32).astype(np.float64)
        rc = O.raycast([ov], og, K, T32, w, h)
        np.testing.assert_array_equal(rc["k"] >= 0, hit)
        kc = O.structure(rc)
        fd = np.zeros(6)
        eps = 1e-6
        for i in range(6):
            e = np.zeros(6)
            e[i] = eps
            zp = O.depth_fixed(ov, og, K, O.compose(T0, O.se3_exp(xi0 + e)), w, h, kc)
            zm = O.depth_fixed(ov, og, K, O.compose(T0, O.se3_exp(xi0 - e)), w, h, kc)
            fd[i] = np.sum(gdm * (zp - zm)) / (2 * eps)
        assert np.linalg.norm(g - fd) / np.linalg.norm(fd) <= 1e-3, (g, fd)
        # the right-perturbation gradient alone is off by more than the bar here
        g_right = ctx.diffray_backward(F, W, og.origin, og.voxel_size, T, K, t(gdm.astype(np.float32)),
                                       t(rc["k"].astype(np.int32))).cpu().numpy()
        assert np.linalg.norm(g_right - fd) / np.linalg.norm(fd) > 1e-2
