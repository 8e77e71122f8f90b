"""The seeded scene generator: frames are a function of (seed, frame index)
alone, whatever the number of rendering threads."""
import hashlib

import numpy as np

from synth import scenes as S


def _digest(frames):
    h = hashlib.sha256()
    for d, c in frames:
        h.update(np.ascontiguousarray(d).tobytes())
        h.update(np.ascontiguousarray(c).tobytes())
    return h.hexdigest()


def test_frames_reproducible_across_threads():
    seq = S.small_room_sequence(seed=1, n_frames=6)
    idx = [0, 2, 3, 5]
    a = _digest(seq.frames(idx, threads=8))
    b = _digest(seq.frames(idx, threads=3))
    c = _digest([seq.frame(i) for i in idx])
    assert a == b == c


def test_noise_seeded_per_frame():
    seq = S.small_room_sequence(seed=1, n_frames=3)
    d0, _ = seq.frame(1)
    clean = S.small_room_sequence(seed=1, n_frames=3, noise=False).frame(1)[0]
    again = S.add_depth_noise(clean, 1, 1)
    np.testing.assert_array_equal(d0, again)
    other = S.add_depth_noise(clean, 1, 2)
    assert np.any(other != again)
    assert np.all((again > 0) == (clean > 0))


def test_device_renderer_matches_host_renderer():
    """The torch renderer (run here on the CPU) reproduces the host
    renderer's noise-free depth and colour exactly."""
    import torch
    from synth.device_render import DeviceRenderer
    for seq in (S.small_room_sequence(seed=1, n_frames=3), S.large_room_sequence(seed=2, n_frames=20)):
        r = DeviceRenderer(seq.scene, seq.K, torch.device("cpu"))
        for i in (0, 2):
            d0, c0, _ = S.render(seq.scene, seq.K, seq.poses[i])
            d1, c1 = r.frame(seq.poses[i], i)
            np.testing.assert_array_equal(d1.numpy(), d0)
            np.testing.assert_array_equal(c1.numpy(), c0)
    # with noise: seeded, reproducible, zero where there is no surface
    r = DeviceRenderer(seq.scene, seq.K, torch.device("cpu"), noise_seed=5)
    a, _ = r.frame(seq.poses[1], 1)
    b, _ = r.frame(seq.poses[1], 1)
    assert torch.equal(a, b)
