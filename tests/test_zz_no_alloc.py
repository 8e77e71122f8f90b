"""The allocation-free differentiable-raycast backward
(mvf_diffray_backward_noalloc) against the allocating entry point: two calls
in a row, the second on a smaller image, each compared with the allocating
call on the same inputs and with the binary64 oracle gradient."""
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


def test_noalloc_backward_equals_allocating_backward(mvf):
    import torch
    seq = S.small_room_sequence(seed=1, noise=False)
    n = 96
    og = O.OGrid((-1.0, -1.0, -1.0), 2.0 / n, 4.0, 128)
    ov = O.OVolume.empty((n, n, n))
    K = seq.K.as_array()
    for i in range(10):
        d, c = seq.frame(i)
        O.integrate(ov, og, d, c, K, seq.poses[i])
    F = t(ov.F32())
    W = torch.from_numpy(ov.W.view(np.int16).copy()).to(dev())
    rng = np.random.default_rng(21)
    with mvf.Context() as ctx:
        # the second call has fewer pixels (and partial blocks) than the first
        for w, h, scale in ((320, 240, 1.0), (200, 150, 0.625)):
            Ks = np.array([K[0] * scale, K[1] * scale, (w - 1) / 2.0, (h - 1) / 2.0], np.float32)
            T = S.perturb_pose(seq.poses[5], rng, 0.02, 2.0)
            T32 = np.asarray(T, np.float32).astype(np.float64)
            log(f"noalloc backward {w}x{h} on 96^3")
            depth, record = ctx.diffray_forward(F, W, og.origin, og.voxel_size, T32, Ks, w, h)
            gd = rng.normal(size=(h, w)).astype(np.float32) * (record.cpu().numpy() >= 0)
            gdt = t(gd)
            gF_a = torch.zeros_like(F)
            gxi_a = ctx.diffray_backward(F, W, og.origin, og.voxel_size, T32, Ks, gdt, record, gF_a)
            gF_b = torch.zeros_like(F)
            gxi_b = ctx.diffray_backward(F, W, og.origin, og.voxel_size, T32, Ks, gdt, record, gF_b, noalloc=True)
            torch.cuda.synchronize()
            ga, gb = gxi_a.cpu().numpy(), gxi_b.cpu().numpy()
            # the pose partials are reduced in a fixed order: identical bits
            np.testing.assert_array_equal(ga.view(np.uint64), gb.view(np.uint64))
            # voxel gradients are float atomics (order-dependent rounding)
            Fa, Fb = gF_a.cpu().numpy().astype(np.float64), gF_b.cpu().numpy().astype(np.float64)
            assert np.abs(Fa).max() > 0
            assert np.abs(Fa - Fb).max() <= 1e-6 * np.abs(Fa).max()
            # and both equal the binary64 oracle gradient at the parity bar
            rc = O.raycast([ov], og, Ks, T32, w, h)
            np.testing.assert_array_equal(record.cpu().numpy(), rc["k"])
            g_ref, gF_ref = O.depth_grad(ov, og, Ks, T32, w, h, O.structure(rc), gd.astype(np.float64))
            assert np.linalg.norm(gb - g_ref) / np.linalg.norm(g_ref) <= 1e-3
            assert np.abs(Fb - gF_ref).max() <= 1e-3 * np.abs(gF_ref).max()


def test_noalloc_backward_rejects_images_beyond_its_scratch(mvf):
    import torch
    from paper_1511_07106_amd import _lib as L
    F = torch.zeros((8, 8, 8), dtype=torch.float32, device=dev())
    W = torch.zeros((8, 8, 8), dtype=torch.int16, device=dev())
    w, h = 2048, 2064  # 128 x 129 blocks of 16x16 > 16384
    record = torch.full((h, w), -1, dtype=torch.int32, device=dev())
    gd = torch.zeros((h, w), dtype=torch.float32, device=dev())
    K = np.array([500.0, 500.0, w / 2, h / 2], np.float32)
    T = S.look_at([0, 0, -1], [0, 0, 0])
    with mvf.Context() as ctx:
        with pytest.raises(L.MvfError) as ei:
            ctx.diffray_backward(F, W, (0, 0, 0), 0.1, T, K, gd, record, None, noalloc=True)
        assert ei.value.status == L.MVF_ERR_INVALID_ARG
        # the allocating entry point takes the same image
        ctx.diffray_backward(F, W, (0, 0, 0), 0.1, T, K, gd, record, None)
        torch.cuda.synchronize()
