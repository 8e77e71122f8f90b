"""The analytic-scene renderer of ``scenes.render`` written with torch tensor
operations, so that workloads of thousands of frames (many independent
rooms, long walks) can be generated directly in device memory.

Input generation only: the same ray/solid intersections as the host
renderer in binary64, then z-depth in binary32.  Depth noise is drawn from
a torch generator seeded by (scene seed, frame) -- seeded and reproducible,
but a different stream from the host renderer's PCG64 noise, so frames from
the two renderers are not interchangeable where noise is on."""
from __future__ import annotations

import numpy as np

from .scenes import Intrinsics, Scene


class DeviceRenderer:
    """Renders frames of one scene at one camera into device tensors."""

    def __init__(self, scene: Scene, K: Intrinsics, device, noise_seed=None, sigma_coeff: float = 0.0015):
        import torch
        self.torch = torch
        self.dev = device
        self.K = K
        self.noise_seed = noise_seed
        self.sigma = sigma_coeff
        u = torch.arange(K.width, dtype=torch.float64, device=device)
        v = torch.arange(K.height, dtype=torch.float64, device=device)
        vv, uu = torch.meshgrid(v, u, indexing="ij")
        self.rays = torch.stack([(uu - K.cx) / K.fx, (vv - K.cy) / K.fy, torch.ones_like(uu)], -1).reshape(-1, 3)
        self.scene = scene
        pal = np.concatenate([scene.wall_colors] + [s.color[None] for s in scene.spheres]
                             + [b.color[None] for b in scene.boxes], axis=0).astype(np.uint8)
        self.palette = torch.from_numpy(pal).to(device)

    def frame(self, T_wc, frame_index: int = 0):
        """(depth f32 (H, W) z-depth in metres, 0 = no surface; rgb u8 (H, W, 3))."""
        torch = self.torch
        sc = self.scene
        T = np.asarray(T_wc, np.float64)
        R = torch.from_numpy(T[:, :3].copy()).to(self.dev)
        C = T[:, 3]
        rc = self.rays
        d = torch.stack([rc[:, 0] * R[a, 0] + rc[:, 1] * R[a, 1] + rc[:, 2] * R[a, 2] for a in range(3)], 1)
        n = d.shape[0]
        inf = torch.tensor(float("inf"), dtype=torch.float64, device=self.dev)
        best = torch.full((n,), float("inf"), dtype=torch.float64, device=self.dev)
        obj = torch.full((n,), -1, dtype=torch.int64, device=self.dev)
        for a in range(3):
            da = d[:, a]
            tpos = (float(sc.room_hi[a]) - float(C[a])) / da
            tneg = (float(sc.room_lo[a]) - float(C[a])) / da
            t = torch.where(da > 0, tpos, torch.where(da < 0, tneg, inf))
            wall = torch.where(da > 0, torch.full_like(obj, 2 * a + 1), torch.full_like(obj, 2 * a))
            m = t < best
            best = torch.where(m, t, best)
            obj = torch.where(m, wall, obj)
        base = 6
        a2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
        for si, s in enumerate(sc.spheres):
            oc = C - s.center
            b = d[:, 0] * float(oc[0]) + d[:, 1] * float(oc[1]) + d[:, 2] * float(oc[2])
            c = float(oc @ oc) - float(s.radius) ** 2
            disc = b * b - a2 * c
            ok = disc >= 0
            sq = torch.sqrt(torch.where(ok, disc, torch.zeros_like(disc)))
            t = (-b - sq) / a2
            m = ok & (t > 1e-9) & (t < best)
            best = torch.where(m, t, best)
            obj = torch.where(m, torch.full_like(obj, base + si), obj)
        base += len(sc.spheres)
        Ct = torch.from_numpy(C.copy()).to(self.dev)
        for bi, bx in enumerate(sc.boxes):
            lo = torch.from_numpy((bx.center - bx.half).copy()).to(self.dev)
            hi = torch.from_numpy((bx.center + bx.half).copy()).to(self.dev)
            t1 = (lo[None, :] - Ct[None, :]) / d
            t2 = (hi[None, :] - Ct[None, :]) / d
            par = d == 0
            inside = ((Ct >= lo) & (Ct <= hi))[None, :].expand_as(d)
            tmin = torch.where(par, torch.where(inside, -inf, inf), torch.minimum(t1, t2))
            tmax = torch.where(par, torch.where(inside, inf, -inf), torch.maximum(t1, t2))
            tn = tmin.max(dim=1).values
            tf = tmax.min(dim=1).values
            m = (tn <= tf) & (tn > 1e-9) & (tn < best)
            best = torch.where(m, tn, best)
            obj = torch.where(m, torch.full_like(obj, base + bi), obj)
        depth = torch.where(torch.isfinite(best), best, torch.zeros_like(best))
        if self.noise_seed is not None:
            g = torch.Generator(device=self.dev)
            g.manual_seed(int(self.noise_seed) * 1000003 + 1000 + int(frame_index))
            noisy = depth + torch.randn(depth.shape, generator=g, dtype=torch.float64, device=self.dev) \
                * self.sigma * depth * depth
            depth = torch.where(depth > 0, torch.clamp(noisy, min=1e-3), torch.zeros_like(depth))
        H, W = self.K.height, self.K.width
        rgb = self.palette[obj.clamp(min=0)].reshape(H, W, 3)
        return depth.to(torch.float32).reshape(H, W).contiguous(), rgb.contiguous()
