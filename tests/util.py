"""Helpers shared by the GPU tests (test side only)."""
import sys

import numpy as np

import oracle as O
from synth import scenes as S


def log(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a fault still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev():
    import torch
    return torch.device("cuda", 0)


def t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def fuse_both(ctx, gid, og, vol_specs, seq, frame_ids, rgb=True, stream_id=0):
    """Create volumes (offset, dims) in the GPU context and the oracle, fuse
    the frames into both, return (gpu volume ids, oracle volumes)."""
    ids = [ctx.volume(gid, off, dims, stream_id=stream_id) for off, dims in vol_specs]
    ovs = [O.OVolume.empty(dims, off) for off, dims in vol_specs]
    K = seq.K.as_array()
    for i in frame_ids:
        d, c = seq.frame(i)
        for ov in ovs:
            O.integrate(ov, og, d, c if rgb else None, K, seq.poses[i])
        ctx.integrate(t(d), t(c) if rgb else None, seq.poses[i], K, stream_id=stream_id)
    return ids, ovs


def compare_volume(ctx, vid, ov, f_tol=1e-5):
    F, W, Cc = ctx.read_volume(vid)
    np.testing.assert_array_equal(W, ov.W)
    np.testing.assert_array_equal(Cc, ov.Cc)
    err = np.abs(F.astype(np.float64) - ov.F)
    assert err.max() <= f_tol, f"max |dF| = {err.max()}"
    return F, W, Cc, float(err.max())


def raycast_both(ctx, ovs, og, K, T, w, h, step=0.5, stream_id=0, F32=None):
    out = ctx.raycast(T, K, w, h, stream_id=stream_id)
    import torch
    torch.cuda.synchronize()
    rc = O.raycast(ovs, og, K, T, w, h, step=step, F32=F32)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    return g, rc


def check_raycast(g, rc, ids, depth_tol=1e-4, normal_tol=2e-3, exact_hits=True):
    """GPU raycast vs oracle: validity and hit volume exact, depth within
    depth_tol, vertex within depth_tol * 2, normal within normal_tol."""
    hit_g = g["hit"] >= 0
    hit_o = rc["hit"] >= 0
    if exact_hits:
        if not np.array_equal(hit_g, hit_o):
            bad = np.argwhere(hit_g != hit_o)
            for (v, u) in bad[:6]:
                print(f"  pixel ({u},{v}): device depth {g['depth'][v, u]!r} hit {g['hit'][v, u]}; oracle "
                      f"k {rc['k'][v, u]} t* {rc['tstar'][v, u]!r} depth {rc['depth'][v, u]!r} "
                      f"amb {rc['ambiguous'][v, u]}", flush=True)
            raise AssertionError(f"validity differs on {len(bad)} pixels (device {int(hit_g.sum())}, "
                                 f"oracle {int(hit_o.sum())})")
        mapped = np.where(hit_o, np.asarray(ids)[np.maximum(rc["hit"], 0)], -1)
        np.testing.assert_array_equal(g["hit"], mapped)
    both = hit_g & hit_o
    assert np.all(g["depth"][~hit_g] == 0)
    if both.any():
        dd = np.abs(g["depth"].astype(np.float64) - rc["depth"])[both]
        assert dd.max() <= depth_tol, f"max |d depth| = {dd.max()}"
        dv = np.abs(g["vertex"].astype(np.float64) - rc["vertex"])[both]
        assert dv.max() <= 2 * depth_tol, f"max |d vertex| = {dv.max()}"
        gn = g["normal"][both].astype(np.float64)
        on = rc["normal"][both]
        ok = np.isfinite(on).all(axis=1)
        dn = np.abs(gn[ok] - on[ok])
        assert dn.size == 0 or dn.max() <= normal_tol, f"max |d normal| = {dn.max()}"
    return int(both.sum())
