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
