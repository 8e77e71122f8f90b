"""Benchmark: TSDF integration voxel-updates/s and raycast Mpix/s on one
MI355X, with the fraction of HBM bandwidth the integration kernel reaches,
and the batched form against the plain per-volume form.

Workload (the KinectFusion-scale equivalence case): synthetic 640x480
depth + RGB frames (fx = fy = 525, cx = 319.5, cy = 239.5) of a 4 m room
with 12 seeded spheres/boxes on a seeded 0.5 m/s handheld path at 30 fps
(300 frames).  One step = one frame: frame preparation, integration into
every active volume, raycast of the frame's pose.  Inputs are rendered on
the host and resident in device memory before the timed region.

Phases (all run by default):
  single       one 512^3 volume over a 3 m cube (5.86 mm voxels), plain
               mvf_integrate + mvf_raycast calls (each kernel timed with HIP
               events: the roofline figures come from here)
  single_step  the same volume through mvf_step (the per-frame sequence
               replayed as a HIP graph); the headline value
  tiled        8 volumes of 257^3 at offsets {0,255}^3 (same voxels), plain
               per-volume calls
  batched      the same 8 volumes through mvf_step (one persistent launch each
               for integration and raycast, replayed as a HIP graph)
  probe        roofline probe (not a workload of the paper): one 512^3 volume
               wholly inside the view in front of a far plane, so that every
               voxel is updated in every frame (1.6 GB of TSDF traffic per
               frame, far above the 256 MB Infinity Cache)
  small        128^3 over 2 m, ten 320x240 frames of the small room, through
               mvf_step and through the plain calls (absolute units only: the
               21 MB volume stays in the Infinity Cache)
  multi        32 independent rooms, 1-4 uneven volumes of 128^3..384^3 each,
               distinct 640x480 frames of each room's 100-frame path; the
               batched step against the rooms' plain calls
  corridor     dynamic placement down a 20 m corridor: volumes of three sizes
               (512^3, 384^3, 256^3) under an 8 GB budget, through mvf_step
               and through the plain calls
  diffray      pose refinement through the differentiable raycast at 512^3
  passing      the memory-passing regime: time per frame against the number of
               512^3 volumes with a device budget of one volume, and resident
  tracking     the per-frame loop with ICP camera tracking against the last
               raycast (the 512^3 large room): time per part and pose error
  table1       surface points of one 512^3 volume vs eight 512^3 volumes over
               the same 3 m cube: point count and distance to the analytic
               surface (the paper's resolution and accuracy metrics)

Prints one JSON line.  python bench.py [--steps K] [--warmup W] [--gpus 1]
[--phases a,b,...] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TSDF voxel-updates/s + raycast Mpix/s at 1 GPU; % HBM peak; batched vs plain"
HBM_PEAK_GBS = 8000.0
N_VOX = 512
EXTENT = 3.0
W_IMG, H_IMG = 640, 480
# algorithmic bytes of the integration kernel: F (4) + W (2) read and written
# per updated voxel, colour (4) read and written per band voxel, and the
# prepared range (4) and colour (4) maps read once per pixel
B_UPDATED, B_BAND, B_PIXEL = 12, 8, 8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1511_07106_amd", "csrc", "mvf_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()


def render_frames(n_frames: int, total: int = 300):
    from synth import scenes as S
    seq = S.large_room_sequence(seed=2, n_frames=total)
    idx = [i % total for i in range(n_frames)]
    t0 = time.time()
    frames = seq.frames(sorted(set(idx)), threads=16)
    by = dict(zip(sorted(set(idx)), frames))
    log(f"rendered {len(by)} frames in {time.time() - t0:.1f}s")
    return seq, [(by[i], seq.poses[i]) for i in idx]


TUNE_STEPS = 120 + 2  # the autotuner's runs (15 blocks of 8: the reference between the 7 others) and two more


def run_phase(mvf, torch, phase, dev_frames, poses, K, warmup, steps, timed=False, tune_cache=None,
              tune=False):
    """Wall-clock run of one phase; with timed=True the library also times
    every kernel launch with events (a separate run: the events themselves
    cost a few microseconds per call).  Batched phases take their launch
    schedule from tune_cache (written by a tuning run with tune=True)."""
    origin = (-EXTENT / 2,) * 3
    s = EXTENT / N_VOX
    ctx = mvf.Context(timing=timed)
    if tune_cache and not tune:
        ctx.autotune("cached", tune_cache)
    gid = ctx.grid(origin, s, 4.0, 128)
    if phase in ("single", "single_step"):
        ctx.volume(gid, (0, 0, 0), (N_VOX,) * 3)
    else:
        h = N_VOX // 2
        for oz in (0, h - 1):
            for oy in (0, h - 1):
                for ox in (0, h - 1):
                    ctx.volume(gid, (ox, oy, oz), (h + 1,) * 3)
    dev = torch.device("cuda", 0)
    out = {"depth": torch.empty((H_IMG, W_IMG), device=dev),
           "vertex": torch.empty((H_IMG, W_IMG, 3), device=dev),
           "normal": torch.empty((H_IMG, W_IMG, 3), device=dev),
           "hit": torch.empty((H_IMG, W_IMG), dtype=torch.int32, device=dev)}

    def one(i):
        d, c = dev_frames[i]
        if phase in ("batched", "single_step"):
            ctx.step([(0, d, c, poses[i], K)], [out])
        else:
            ctx.integrate(d, c, poses[i], K)
            ctx.raycast(poses[i], K, W_IMG, H_IMG, out=out)

    if tune:
        # tune on the frames the timed run sees, after the same warm-up
        for i in range(warmup):
            one(i)
        ctx.autotune("tune", tune_cache)
        for i in range(warmup, warmup + TUNE_STEPS):
            one(i % len(dev_frames))
        torch.cuda.synchronize()
        sched = ctx.schedule()
        ctx.close()
        return sched
    for i in range(warmup):
        one(i)
    torch.cuda.synchronize()
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        one(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    hit_frac = float((out["depth"] > 0).float().mean())
    sched = ctx.schedule() if phase in ("batched", "single_step") else None
    ctx.close()
    r = {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "voxels_updated": st["voxels_updated"],
         "voxels_band": st["voxels_band"], "integrate_ms": st["integrate_ms"], "raycast_ms": st["raycast_ms"],
         "step_ms": st["step_ms"], "integrate_launches": st["integrate_launches"],
         "raycast_launches": st["raycast_launches"], "hit_fraction_last": hit_frac,
         "bricks_projected_per_step": st["bricks_projected"] / steps, "bricks_deep_per_step": st["bricks_deep"] / steps}
    if sched:
        r["schedule"] = sched
    r["voxel_updates_per_s"] = st["voxels_updated"] / wall
    r["raycast_mpix_s"] = steps * W_IMG * H_IMG / wall / 1e6
    if st["integrate_ms"] > 0:
        r["integrate_kernel_voxel_updates_per_s"] = st["voxels_updated"] / (st["integrate_ms"] * 1e-3)
    if st["raycast_ms"] > 0:
        r["raycast_kernel_mpix_s"] = steps * W_IMG * H_IMG / (st["raycast_ms"] * 1e-3) / 1e6
    return r


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def phase_probe(mvf, torch, steps=60, warmup=5):
    """Roofline probe: one 512^3 volume over 3 m seen from 3.6 m in front of
    its near face (wholly inside the 640x480 view), and a depth map of a
    fronto-parallel plane 7.5 m away behind it: every voxel is in front of
    the surface and within the view, so all 134 M voxels are updated (F and
    W read and written) in every frame and no colour band exists."""
    dev = torch.device("cuda", 0)
    s = EXTENT / N_VOX
    T = np.zeros((3, 4))
    T[:, :3] = np.eye(3)
    T[:, 3] = [0.0, 0.0, -EXTENT / 2 - 3.6]
    depth = torch.full((H_IMG, W_IMG), 7.5, dtype=torch.float32, device=dev)
    rgb = torch.zeros((H_IMG, W_IMG, 3), dtype=torch.uint8, device=dev)
    K = np.array([525.0, 525.0, 319.5, 239.5], np.float32)
    res = {}
    for timed in (False, True):
        with mvf.Context(timing=timed) as ctx:
            gid = ctx.grid((-EXTENT / 2,) * 3, s, 4.0, 128)
            ctx.volume(gid, (0, 0, 0), (N_VOX,) * 3)
            for _ in range(warmup):
                ctx.integrate(depth, rgb, T, K)
            torch.cuda.synchronize()
            ctx.reset_stats()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.integrate(depth, rgb, T, K)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = ctx.stats()
        if not timed:
            res["ms_per_frame"] = 1e3 * wall / steps
            res["voxel_updates_per_frame"] = st["voxels_updated"] / steps
            res["voxel_updates_per_s"] = st["voxels_updated"] / wall
        else:
            avg_s = st["integrate_ms"] * 1e-3 / max(1, st["integrate_launches"])
            bytes_launch = (B_UPDATED * st["voxels_updated"] + B_BAND * st["voxels_band"]) / steps \
                + B_PIXEL * W_IMG * H_IMG
            res["integrate_avg_launch_ms"] = avg_s * 1e3
            res["algorithmic_bytes_per_launch"] = bytes_launch
            res["achieved_gb_s"] = bytes_launch / avg_s / 1e9
            res["frac"] = res["achieved_gb_s"] / HBM_PEAK_GBS
    res["all_voxels_updated"] = res["voxel_updates_per_frame"] == float(N_VOX ** 3)
    return res


def phase_small(mvf, torch, reps=6, warmup=1):
    """The plain single-volume case: 128^3 over [-1, 1]^3 (15.6 mm voxels),
    the ten 320x240 frames of the small room (3 spheres) on its 1 m circle;
    each step integrates one frame and raycasts its view.  The ten frames are
    replayed `reps` times after `warmup` passes (each pass fuses them again),
    through mvf_step (a graph replay per frame) and through the plain calls."""
    from synth import scenes as S
    seq = S.small_room_sequence(seed=1)
    K = seq.K.as_array()
    w, h = seq.K.width, seq.K.height
    dev = torch.device("cuda", 0)
    fr = [(torch.from_numpy(d).to(dev), torch.from_numpy(c).to(dev)) for d, c in seq.frames(range(10), threads=10)]
    res = {"volume": [128, 128, 128], "image": [w, h], "frames": 10}
    for path in ("step", "plain"):
        with mvf.Context() as ctx:
            gid = ctx.grid((-1.0,) * 3, 2.0 / 128, 4.0, 128)
            ctx.volume(gid, (0, 0, 0), (128,) * 3)
            out = {"depth": torch.empty((h, w), device=dev), "vertex": torch.empty((h, w, 3), device=dev),
                   "normal": torch.empty((h, w, 3), device=dev),
                   "hit": torch.empty((h, w), dtype=torch.int32, device=dev)}

            def one(i):
                d, c = fr[i]
                if path == "step":
                    ctx.step([(0, d, c, seq.poses[i], K)], [out])
                else:
                    ctx.integrate(d, c, seq.poses[i], K)
                    ctx.raycast(seq.poses[i], K, w, h, out=out)

            for _ in range(warmup):
                for i in range(10):
                    one(i)
            torch.cuda.synchronize()
            ctx.reset_stats()
            t0 = time.perf_counter()
            for _ in range(reps):
                for i in range(10):
                    one(i)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            st = ctx.stats()
        n = 10 * reps
        res[path] = {"ms_per_step": 1e3 * wall / n, "voxel_updates_per_s": st["voxels_updated"] / wall,
                     "raycast_mpix_s": n * w * h / wall / 1e6}
    return res


def phase_diffray(mvf, torch, n_poses=16, n_steps=50):
    """Pose refinement through the differentiable raycast: a 512^3 volume over
    [-1, 1]^3 fused from 60 noisy 640x480 frames of the small room on its
    circle; 16 poses perturbed by 2 cm / 2 degrees, 50 gradient steps each
    against the noise-free analytic depth at the true pose."""
    from synth import scenes as S
    from paper_1511_07106_amd.autograd import DiffRaycast, depth_loss
    n = 512
    seq = S.small_room_sequence(seed=1, n_frames=60, K=S.K_VGA)
    K = seq.K.as_array()
    dev = torch.device("cuda", 0)
    t0 = time.time()
    frames = seq.frames(list(range(60)), threads=16)
    with mvf.Context() as ctx:
        gid = ctx.grid((-1.0, -1.0, -1.0), 2.0 / n, 4.0, 128)
        vid = ctx.volume(gid, (0, 0, 0), (n, n, n))
        for i, (d, c) in enumerate(frames):
            ctx.integrate(torch.from_numpy(d).to(dev), torch.from_numpy(c).to(dev), seq.poses[i], K)
        ctx.synchronize()
        # the plain raycast of the same volume at the same (perturbed) poses,
        # timed the same way as the differentiable forward below
        rng_p = np.random.default_rng(5)
        plain_ms = []
        for pi in [int(x) for x in np.linspace(0, 59, n_poses)]:
            Tp = S.perturb_pose(seq.poses[pi], rng_p, 0.02, 2.0)
            for _ in range(4):
                a, b = _events(torch)
                a.record()
                ctx.raycast(Tp, K, W_IMG, H_IMG)
                b.record()
                torch.cuda.synchronize()
                plain_ms.append(a.elapsed_time(b))
        F_np, W_np, _ = ctx.read_volume(vid)
    F = torch.from_numpy(F_np).to(dev)
    W = torch.from_numpy(W_np.view(np.int16)).to(dev)
    del F_np, W_np
    log(f"diffray: fused 60 frames into 512^3 in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(5)
    pose_idx = [int(x) for x in np.linspace(0, 59, n_poses)]
    fwd_ms, bwd_ms, err0, err1, rot0, rot1, loss_ratio = [], [], [], [], [], [], []

    def rot_err(A, B):
        R = A[:, :3].T @ B[:, :3]
        return float(np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))))

    with mvf.Context() as ctx:
        for pi in pose_idx:
            T_true = seq.poses[pi]
            target = torch.from_numpy(S.render(seq.scene, seq.K, T_true)[0]).to(dev)
            T = S.perturb_pose(T_true, rng, 0.02, 2.0)
            err0.append(float(np.linalg.norm(T[:, 3] - T_true[:, 3])))
            rot0.append(rot_err(T, T_true))
            losses = []
            for it in range(n_steps):
                xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
                a, b = _events(torch)
                a.record()
                # F and W stay fixed: generation 1 keeps the library's copy
                depth = DiffRaycast.apply(F, xi, W, ctx, (-1.0, -1.0, -1.0), 2.0 / n, T, K, W_IMG, H_IMG, 1)
                b.record()
                loss = depth_loss(depth, target)
                c_, d_ = _events(torch)
                c_.record()
                loss.backward()
                d_.record()
                torch.cuda.synchronize()
                fwd_ms.append(a.elapsed_time(b))
                bwd_ms.append(c_.elapsed_time(d_))
                losses.append(float(loss))
                T = mvf.pose_retract(T, -0.5 * xi.grad.numpy())
            err1.append(float(np.linalg.norm(T[:, 3] - T_true[:, 3])))
            rot1.append(rot_err(T, T_true))
            loss_ratio.append(losses[-1] / max(losses[0], 1e-30))
    return {"poses": n_poses, "steps": n_steps, "image": [W_IMG, H_IMG], "volume": [n, n, n],
            "forward_ms_median": float(np.median(fwd_ms)), "backward_ms_median": float(np.median(bwd_ms)),
            "backward_over_forward": float(np.median(bwd_ms) / np.median(fwd_ms)),
            "plain_raycast_ms_median": float(np.median(plain_ms)),
            "forward_over_plain_raycast": float(np.median(fwd_ms) / np.median(plain_ms)),
            "trans_err_mm_before": 1e3 * float(np.mean(err0)), "trans_err_mm_after": 1e3 * float(np.mean(err1)),
            "rot_err_deg_before": float(np.mean(rot0)), "rot_err_deg_after": float(np.mean(rot1)),
            "loss_ratio_median": float(np.median(loss_ratio)),
            "poses_improved": int(sum(e1 < e0 for e0, e1 in zip(err0, err1)))}


def phase_multi(mvf, torch, n_rooms=32, n_frames=100, warmup=10):
    """Many independent scenes: 32 rooms with 1-4 volumes of 128^3..384^3 each
    (10.4 mm voxels), each room streaming the distinct 640x480 frames of its
    own 100-frame handheld path (rendered into device memory); one step takes
    one frame of every room.  The batched step (all rooms in one mvf_step,
    autotuned schedule) against the 32 rooms' plain per-volume calls, over
    frames warmup..n_frames-1 of every path after the first `warmup`."""
    from synth import scenes as S
    from synth.device_render import DeviceRenderer
    s = 4.0 / 384
    rooms = S.multi_room_workload(n_rooms, n_frames)
    dev = torch.device("cuda", 0)
    t0 = time.time()
    frames = []
    for r in rooms:
        rd = DeviceRenderer(r.scene, r.K, dev, noise_seed=r.seed)
        frames.append([rd.frame(r.poses[i], i) for i in range(n_frames)])
    torch.cuda.synchronize()
    log(f"multi: rendered {n_rooms * n_frames} frames on the device in {time.time() - t0:.1f}s")
    K = S.K_VGA.as_array()
    res = {}
    cache = os.path.join(tempfile.mkdtemp(prefix="mvf_tune_"), "schedules.jsonl")
    steps = n_frames - warmup
    for mode in ("tune", "batched", "plain"):
        with mvf.Context(timing=False) as ctx:
            if mode != "plain":
                # the batched form's schedule: tuned on a separate context first
                ctx.autotune("tune" if mode == "tune" else "cached", cache)
            gid = ctx.grid((-2.0, -2.0, -2.0), s, 4.0, 128)
            nvol = 0
            vox = 0
            for i in range(n_rooms):
                for off, dims in S.room_volumes(1000 + i, s):
                    ctx.volume(gid, off, dims, stream_id=i)
                    nvol += 1
                    vox += dims[0] * dims[1] * dims[2]
            outs = [{"depth": torch.empty((H_IMG, W_IMG), device=dev),
                     "vertex": torch.empty((H_IMG, W_IMG, 3), device=dev),
                     "normal": torch.empty((H_IMG, W_IMG, 3), device=dev),
                     "hit": torch.empty((H_IMG, W_IMG), dtype=torch.int32, device=dev)} for _ in range(n_rooms)]

            def one(j):
                fi = j % n_frames
                if mode != "plain":
                    ctx.step([(i, frames[i][fi][0], frames[i][fi][1], rooms[i].poses[fi], K)
                              for i in range(n_rooms)], outs)
                else:
                    for i in range(n_rooms):
                        ctx.integrate(frames[i][fi][0], frames[i][fi][1], rooms[i].poses[fi], K, stream_id=i)
                        ctx.raycast(rooms[i].poses[fi], K, W_IMG, H_IMG, stream_id=i, out=outs[i])

            if mode == "tune":
                for j in range(TUNE_STEPS):
                    one(j)
                torch.cuda.synchronize()
                res["schedule"] = ctx.schedule()
                continue
            for j in range(warmup):
                one(j)
            torch.cuda.synchronize()
            ctx.reset_stats()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for j in range(warmup, n_frames):
                one(j)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            st = ctx.stats()
            res[mode] = {"ms_per_step": 1e3 * wall / steps, "voxel_updates_per_s": st["voxels_updated"] / wall,
                         "mpix_s": steps * n_rooms * W_IMG * H_IMG / wall / 1e6}
            res["volumes"] = nvol
            res["voxels"] = vox
    del frames
    res["rooms"] = n_rooms
    res["frames_per_room"] = n_frames
    res["timed_steps"] = steps
    res["batched_vs_plain_speedup"] = res["plain"]["ms_per_step"] / res["batched"]["ms_per_step"]
    return res


CORRIDOR_CLASSES = [(512, 4), (384, 6), (256, 6)]


def phase_corridor(mvf, torch, n_steps=40, stride=10, classes=CORRIDOR_CLASSES, budget_gb=8.0):
    """Dynamic placement down the 20 m corridor: every `stride`-th frame of the
    2000-frame walk is integrated into the live volumes and raycast in one
    mvf_step (one graph replay, or one per wave when the live volumes exceed
    the budget), then the endpoint-count placement adds/removes volumes of
    three sizes (512^3, 384^3, 256^3 at 2.93 mm: 1.5, 1.125 and 0.75 m; at
    most 4, 6 and 6 live, the largest taking the highest-count regions,
    beta 1.5) under an 8 GB device budget (16 live volumes need 9.8 GB), so
    that volumes swap to and from host memory.  The same walk through the
    plain calls is timed beside it."""
    from synth import scenes as S
    seq = S.corridor_sequence(seed=3, n_frames=2000)
    K = seq.K.as_array()
    idx = [i * stride for i in range(n_steps)]
    dev = torch.device("cuda", 0)
    t0 = time.time()
    fr = seq.frames(idx, threads=16)
    frames = [(torch.from_numpy(d).to(dev), torch.from_numpy(c).to(dev)) for d, c in fr]
    log(f"corridor: rendered {len(idx)} frames in {time.time() - t0:.1f}s")
    out = {"depth": torch.empty((H_IMG, W_IMG), device=dev),
           "vertex": torch.empty((H_IMG, W_IMG, 3), device=dev),
           "normal": torch.empty((H_IMG, W_IMG, 3), device=dev),
           "hit": torch.empty((H_IMG, W_IMG), dtype=torch.int32, device=dev)}
    res = {"steps": n_steps, "frame_stride": stride, "classes": [list(c) for c in classes], "budget_gb": budget_gb}
    for path in ("step", "plain"):
        with mvf.Context(budget_bytes=int(budget_gb * (1 << 30)), timing=False) as ctx:
            gid = ctx.grid((0.0, -1.0, 0.0), 0.00293, 4.0, 128)
            added = removed = 0
            hits = []
            place_ms = []
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for j, i in enumerate(idx):
                d, c = frames[j]
                if path == "step":
                    ctx.step([(0, d, c, seq.poses[i], K)], [out])
                else:
                    ctx.integrate(d, c, seq.poses[i], K)
                    ctx.raycast(seq.poses[i], K, W_IMG, H_IMG, out=out)
                tp = time.perf_counter()
                a, r, _ = ctx.placement_update_classes(d, seq.poses[i], K, gid, classes, 1.5)
                place_ms.append(1e3 * (time.perf_counter() - tp))
                added += len(a)
                removed += len(r)
                if j % 10 == 9:
                    hits.append(float((out["depth"] > 0).float().mean()))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            st = ctx.stats()
        res[path] = {"ms_per_step": 1e3 * wall / n_steps, "placement_ms_median": float(np.median(place_ms)),
                     "volumes_added": added, "volumes_removed": removed,
                     "swaps_in": st["swaps_in"], "swaps_out": st["swaps_out"],
                     "h2d_gb": st["bytes_h2d"] / 1e9, "d2h_gb": st["bytes_d2h"] / 1e9,
                     "swap_gb_per_s_of_wall": (st["bytes_h2d"] + st["bytes_d2h"]) / 1e9 / wall,
                     "voxel_updates_per_s": st["voxels_updated"] / wall, "hit_fraction_mean": float(np.mean(hits))}
        log(f"corridor {path}: {res[path]['ms_per_step']:.2f} ms per step")
    res["batched_vs_plain_speedup"] = res["plain"]["ms_per_step"] / res["step"]["ms_per_step"]
    return res


def phase_table1(mvf, torch, n_frames=90):
    """A synthetic stand-in for the paper's single-volume vs eight-volume
    comparison: the large room's first n_frames 640x480 frames (device
    rendered, noisy) fused into one 512^3 volume over the 3 m cube (5.86 mm
    voxels; its 511 cells span 3 m) and into eight 512^3 volumes of 1.5 m
    forming the same cube (2.94 mm voxels, neighbours sharing one voxel
    layer, so every cell lies in exactly one volume).  Surface points of every volume are extracted
    on the device; resolution = point count, accuracy = distance of each
    point to the analytic scene surface (mean, median, standard deviation)."""
    from synth import scenes as S
    from synth.device_render import DeviceRenderer
    seq = S.large_room_sequence(seed=2, noise=True)
    K = seq.K.as_array()
    dev = torch.device("cuda", 0)
    rd = DeviceRenderer(seq.scene, seq.K, dev, noise_seed=seq.seed)
    frames = [rd.frame(seq.poses[i], i) for i in range(n_frames)]
    res = {"frames": n_frames, "image": [W_IMG, H_IMG]}
    for name, n_side, s in (("single_512", 1, EXTENT / (N_VOX - 1)), ("eight_512", 2, EXTENT / (2 * N_VOX - 2))):
        with mvf.Context() as ctx:
            gid = ctx.grid((-EXTENT / 2,) * 3, s, 4.0, 128)
            ids = [ctx.volume(gid, (ox * (N_VOX - 1), oy * (N_VOX - 1), oz * (N_VOX - 1)), (N_VOX,) * 3)
                   for oz in range(n_side) for oy in range(n_side) for ox in range(n_side)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i, (d, c) in enumerate(frames):
                ctx.integrate(d, c, seq.poses[i], K)
            torch.cuda.synchronize()
            t_fuse = time.perf_counter() - t0
            t0 = time.perf_counter()
            pts = [ctx.extract(v, with_index=False) for v in ids]
            torch.cuda.synchronize()
            t_extract = time.perf_counter() - t0
            V = np.concatenate([p["V"].cpu().numpy() for p in pts]).astype(np.float64)
        dist = np.abs(S.scene_sdf(seq.scene, V))
        res[name] = {"volumes": len(ids), "voxel_mm": 1e3 * s, "vertices": int(V.shape[0]),
                     "mean_mm": 1e3 * float(dist.mean()), "median_mm": 1e3 * float(np.median(dist)),
                     "std_mm": 1e3 * float(dist.std()), "fuse_ms_per_frame": 1e3 * t_fuse / n_frames,
                     "extract_ms": 1e3 * t_extract}
        log(f"table1 {name}: {V.shape[0]} points, mean {res[name]['mean_mm']:.2f} mm")
        del pts, V, dist
    del frames
    res["vertex_ratio"] = res["eight_512"]["vertices"] / max(1, res["single_512"]["vertices"])
    return res


def phase_passing(mvf, torch, counts=(1, 2, 4, 8, 16), frames=6, warmup=3):
    """The paper's memory-passing regime (its runtime experiment): N volumes of
    512^3 (1.5 m, 2.93 mm voxels) in a 4 x 2 x 2 block in front of the camera,
    all in view, every voxel in front of a far plane and so updated in every
    frame, through mvf_step with a device budget of one volume (every volume
    is uploaded, integrated, raycast and downloaded on every frame, in waves
    of one) and with no budget (all resident).  Time per frame against N."""
    dev = torch.device("cuda", 0)
    s = 1.5 / N_VOX
    T = np.zeros((3, 4))
    T[:, :3] = np.eye(3)
    T[:, 3] = [0.0, 0.0, -3.5]
    K = np.array([525.0, 525.0, 319.5, 239.5], np.float32)
    depth = torch.full((H_IMG, W_IMG), 8.0, dtype=torch.float32, device=dev)
    rgb = torch.zeros((H_IMG, W_IMG, 3), dtype=torch.uint8, device=dev)
    offs = [(ix * N_VOX, iy * N_VOX, iz * N_VOX) for iz in range(2) for iy in range(2) for ix in range(4)]
    out = {"depth": torch.empty((H_IMG, W_IMG), device=dev),
           "vertex": torch.empty((H_IMG, W_IMG, 3), device=dev),
           "normal": torch.empty((H_IMG, W_IMG, 3), device=dev),
           "hit": torch.empty((H_IMG, W_IMG), dtype=torch.int32, device=dev)}
    res = {"volume": [N_VOX] * 3, "volume_gb": None, "frames": frames, "path": "mvf_step", "rows": []}
    for n in counts:
        row = {"volumes": n}
        for mode in ("budget_one_volume", "resident"):
            with mvf.Context(timing=False) as ctx:
                gid = ctx.grid((-3.0, -1.5, 0.0), s, 4.0, 128)
                ids = [ctx.volume(gid, o, (N_VOX,) * 3) for o in offs[:n]]
                vbytes = ctx.query(ids[0])[1]
                res["volume_gb"] = vbytes / 1e9
                if mode == "budget_one_volume":
                    ctx.set_budget(vbytes)
                for _ in range(warmup):
                    ctx.step([(0, depth, rgb, T, K)], [out])
                torch.cuda.synchronize()
                ctx.reset_stats()
                t0 = time.perf_counter()
                for _ in range(frames):
                    ctx.step([(0, depth, rgb, T, K)], [out])
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                st = ctx.stats()
            row[mode] = {"ms_per_frame": 1e3 * wall / frames,
                         "voxel_updates_per_frame": st["voxels_updated"] / frames,
                         "h2d_gb_per_frame": st["bytes_h2d"] / 1e9 / frames,
                         "d2h_gb_per_frame": st["bytes_d2h"] / 1e9 / frames,
                         "swap_gb_per_s": (st["bytes_h2d"] + st["bytes_d2h"]) / 1e9 / wall}
        log(f"passing {n} volumes: {row['budget_one_volume']['ms_per_frame']:.1f} ms per frame with one "
            f"volume's budget, {row['resident']['ms_per_frame']:.2f} ms resident")
        res["rows"].append(row)
    # least-squares slope of time per frame against N
    ns = np.array([r["volumes"] for r in res["rows"]], np.float64)
    for mode in ("budget_one_volume", "resident"):
        ts = np.array([r[mode]["ms_per_frame"] for r in res["rows"]])
        res[f"{mode}_ms_per_added_volume"] = float(np.polyfit(ns, ts, 1)[0])
    return res


def phase_tracking(mvf, torch, n_frames=100):
    """The per-frame loop with tracking (the paper's Fig. 4 order): each new
    640x480 frame of the large room (device rendered, noisy) is tracked by
    ICP against the raycast of the previous pose, then fused into the 512^3
    volume at the tracked pose and raycast there for the next frame.  Reports
    the time of each part and the tracked trajectory's error against the
    true poses (frame 0 is fused at its true pose)."""
    from synth import scenes as S
    from synth.device_render import DeviceRenderer
    seq = S.large_room_sequence(seed=2, noise=True)
    K = seq.K.as_array()
    dev = torch.device("cuda", 0)
    rd = DeviceRenderer(seq.scene, seq.K, dev, noise_seed=seq.seed)
    frames = [rd.frame(seq.poses[i], i) for i in range(n_frames)]

    def outs():
        return {"depth": torch.empty((H_IMG, W_IMG), device=dev),
                "vertex": torch.empty((H_IMG, W_IMG, 3), device=dev),
                "normal": torch.empty((H_IMG, W_IMG, 3), device=dev),
                "hit": torch.empty((H_IMG, W_IMG), dtype=torch.int32, device=dev)}

    maps = [outs(), outs()]
    err_t, err_r, t_track, t_rest, pairs = [], [], [], [], []
    with mvf.Context() as ctx:
        gid = ctx.grid((-EXTENT / 2,) * 3, EXTENT / N_VOX, 4.0, 128)
        ctx.volume(gid, (0, 0, 0), (N_VOX,) * 3)
        T = seq.poses[0]
        ctx.integrate(frames[0][0], frames[0][1], T, K)
        ctx.raycast(T, K, W_IMG, H_IMG, out=maps[0])
        torch.cuda.synchronize()
        for i in range(1, n_frames):
            d, c = frames[i]
            t0 = time.perf_counter()
            T_new, st = ctx.track(d, K, maps[(i - 1) % 2], T, T)
            t1 = time.perf_counter()
            ctx.integrate(d, c, T_new, K)
            ctx.raycast(T_new, K, W_IMG, H_IMG, out=maps[i % 2])
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            T = T_new
            t_track.append(1e3 * (t1 - t0))
            t_rest.append(1e3 * (t2 - t1))
            pairs.append(st["pairs"][-1])
            Tg = seq.poses[i]
            err_t.append(1e3 * float(np.linalg.norm(T[:, 3] - Tg[:, 3])))
            R = T[:, :3].T @ Tg[:, :3]
            err_r.append(float(np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))))
    return {"frames": n_frames, "iters": [10, 5, 4], "track_ms_median": float(np.median(t_track)),
            "trans_err_mm_first5": [round(e, 3) for e in err_t[:5]],
            "integrate_raycast_ms_median": float(np.median(t_rest)),
            "trans_err_mm_mean": float(np.mean(err_t)), "trans_err_mm_max": float(np.max(err_t)),
            "trans_err_mm_last": err_t[-1], "rot_err_deg_mean": float(np.mean(err_r)),
            "rot_err_deg_max": float(np.max(err_r)), "pairs_median": float(np.median(pairs))}


EXTRA_PHASES = {"probe": phase_probe, "small": phase_small, "multi": phase_multi, "corridor": phase_corridor,
                "diffray": phase_diffray, "table1": phase_table1, "passing": phase_passing,
                "tracking": phase_tracking}
DEFAULT_PHASES = "single,single_step,tiled,batched,probe,small,multi,corridor,diffray,table1,passing,tracking"


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seq_frames, K, budget_s=12.0, max_frames=40, threads=None):
    """The CPU oracle on a bounded sample of the same workload: whole steps
    (integrate + raycast) into a 512^3 volume, from the first frame, until
    budget_s of wall time has passed (at least 2 steps), on `threads` host
    threads (default: all the oracle's OpenMP threads)."""
    import oracle as O
    lib = O.lib()
    all_threads = int(lib.orc_threads())
    lib.orc_set_threads(threads or all_threads)
    used = int(lib.orc_threads())
    og = O.OGrid((-EXTENT / 2,) * 3, EXTENT / N_VOX, 4.0, 128)
    ov = O.OVolume.empty((N_VOX,) * 3)
    upd = 0
    n = 0
    t_int = t_ray = 0.0
    t0 = time.perf_counter()
    for (d, c), T in seq_frames[:max_frames]:
        a = time.perf_counter()
        st = O.integrate(ov, og, d, c, K, T)
        b = time.perf_counter()
        upd += st[1]
        O.raycast([ov], og, K, T, W_IMG, H_IMG)
        t_int += b - a
        t_ray += time.perf_counter() - b
        n += 1
        if n >= 2 and time.perf_counter() - t0 > budget_s:
            break
    wall = time.perf_counter() - t0
    lib.orc_set_threads(all_threads)
    return {"value": upd / wall, "unit": "voxel-updates/s", "cores": used, "kind": "oracle",
            "integrate_voxel_updates_per_s": upd / t_int, "raycast_mpix_s": n * W_IMG * H_IMG / t_ray / 1e6,
            "cpu_model": cpu_model(),
            "sample": f"first {n} frames of the timed sequence, integrate + raycast each, into the 512^3 "
                      f"volume on {used} thread(s); {upd} voxel updates in {wall:.1f} s"}


PMC_SUMMARY = os.path.join(ROOT, "profiles", "integrate_kernel_large_room_512_pmc.md")


def traffic_from_profile():
    """HBM bytes per integration launch from the committed rocprofv3 counter
    summary (its 'hbm_bytes_per_dispatch:' line), if that summary was taken
    on the current kernel source ('kernel_source_sha256:' line); else None."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    fields = {}
    for line in open(PMC_SUMMARY):
        if ":" in line and line.split(":", 1)[0].strip() in ("hbm_bytes_per_dispatch", "kernel_source_sha256"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def config_summary(phases):
    """The key figures of every workload, by the configuration it stands for."""
    out = {}
    g = phases.get
    if g("small"):
        out["small_room_128"] = {"step": g("small")["step"], "plain": g("small")["plain"]}
    if g("single_step") or g("single"):
        e = {}
        for k in ("single_step", "single"):
            if g(k):
                e[k] = {x: g(k)[x] for x in ("ms_per_step", "voxel_updates_per_s", "raycast_mpix_s")}
        out["large_room_512"] = e
    if g("tiled") or g("batched"):
        e = {}
        for k in ("tiled", "batched"):
            if g(k):
                e[k] = {x: g(k)[x] for x in ("ms_per_step", "voxel_updates_per_s", "raycast_mpix_s")}
        if g("tiled") and g("batched"):
            e["batched_vs_plain_speedup"] = g("tiled")["ms_per_step"] / g("batched")["ms_per_step"]
        out["large_room_8x257"] = e
    if g("corridor"):
        out["corridor"] = g("corridor")
    if g("multi"):
        m = g("multi")
        out["multi_room_32"] = {k: m[k] for k in ("batched", "plain", "batched_vs_plain_speedup", "volumes")}
    if g("diffray"):
        out["diffray_512"] = g("diffray")
    if g("probe"):
        out["roofline_probe_512"] = g("probe")
    if g("table1"):
        out["surface_points_single_vs_eight"] = g("table1")
    if g("passing"):
        out["memory_passing_sweep"] = g("passing")
    if g("tracking"):
        out["tracked_large_room_512"] = g("tracking")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--phases", default=DEFAULT_PHASES, help="comma list of phases (default: all)")
    ap.add_argument("--schedule-cache", default=None,
                    help="path prefix of the captured phases' schedule files: read when present (no tuning), "
                         "else tuned and written (to profile a run with the schedule of an unprofiled one)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the phases, copy a buffer of this size 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1511_07106_amd as mvf
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    mvf._lib.load()
    from synth import scenes as S
    K = S.K_VGA.as_array()
    dev = torch.device("cuda", 0)
    names = args.phases.split(",")
    frames, dev_frames, poses = [], [], []
    if any(ph not in EXTRA_PHASES for ph in names) or not args.no_cpu:
        # the tuning runs see the frames after the warm-up too: render enough
        # for both
        seq, frames = render_frames(args.warmup + max(args.steps, TUNE_STEPS))
        dev_frames = [(torch.from_numpy(d).to(dev), torch.from_numpy(c).to(dev)) for (d, c), _ in frames]
        poses = [T for _, T in frames]
    torch.cuda.synchronize()
    phases = {}
    for ph in names:
        log(f"phase {ph}")
        if ph in EXTRA_PHASES:
            phases[ph] = EXTRA_PHASES[ph](mvf, torch)
        else:
            cache = None
            if ph in ("single_step", "batched"):
                # the batched form's autotuner picks the launch schedule on a
                # separate context first (untimed), unless a schedule file of
                # an earlier run is given
                if args.schedule_cache:
                    cache = f"{args.schedule_cache}_{ph}.jsonl"
                else:
                    cache = os.path.join(tempfile.mkdtemp(prefix="mvf_tune_"), "schedules.jsonl")
                if not os.path.exists(cache):
                    run_phase(mvf, torch, ph, dev_frames, poses, K, args.warmup, args.steps, tune_cache=cache,
                              tune=True)
            phases[ph] = run_phase(mvf, torch, ph, dev_frames, poses, K, args.warmup, args.steps,
                                   tune_cache=cache)
            if ph in ("single", "tiled"):
                # per-kernel durations from a second, event-timed run of the same frames
                t = run_phase(mvf, torch, ph, dev_frames, poses, K, args.warmup, args.steps, timed=True)
                for k in ("integrate_ms", "raycast_ms", "integrate_launches", "raycast_launches",
                          "integrate_kernel_voxel_updates_per_s", "raycast_kernel_mpix_s"):
                    if k in t:
                        phases[ph][k] = t[k]
                phases[ph]["timed_run_ms_per_step"] = t["ms_per_step"]
        log(json.dumps(phases[ph]))
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 5 copies of {args.copy_probe_mib} MiB")
        del a, b
    # the device's measured copy bandwidth (a 1 GiB device-to-device copy,
    # read plus write, median of 5, HIP events on the current stream): the
    # practical ceiling beside the 8 TB/s specification
    copy_gb_s = None
    try:
        n = (1 << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        copy_gb_s = 2 * (1 << 30) / sorted(ts)[2] / 1e9
        del a, b
    except RuntimeError:
        pass
    # headline: the single 512^3 volume through the graph path; the roofline
    # comes from the plain phase, whose kernels are timed one by one
    core = {k: v for k, v in phases.items() if k not in EXTRA_PHASES}
    if not core:
        print(json.dumps({"phases": phases}), flush=True)
        return
    head_ph = core.get("single_step") or core.get("single") or next(iter(core.values()))
    main_ph = core.get("single") or head_ph
    steps = args.steps
    # roofline of the integration kernel
    upd, band = main_ph["voxels_updated"], main_ph["voxels_band"]
    # the graph path counts no launches of its own: one integration launch per step
    launches = main_ph["integrate_launches"] or steps
    bytes_per_launch = (B_UPDATED * upd + B_BAND * band + B_PIXEL * W_IMG * H_IMG * steps) / launches
    achieved = None
    if main_ph["integrate_ms"] > 0:
        avg_s = main_ph["integrate_ms"] * 1e-3 / launches
        achieved = bytes_per_launch / avg_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic_from_profile(),
            "kernel": "mvf_integrate_kernel", "algorithmic_bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": main_ph["integrate_ms"] / launches if main_ph["integrate_ms"] else None,
            "measured_copy_gb_s": copy_gb_s,
            "frac_of_measured_copy": (achieved / copy_gb_s) if achieved and copy_gb_s else None}
    if "probe" in phases:
        pr = phases["probe"]
        roof["probe_full_frustum"] = {"achieved": pr["achieved_gb_s"], "frac": pr["frac"],
                                      "frac_of_measured_copy": (pr["achieved_gb_s"] / copy_gb_s) if copy_gb_s else None,
                                      "algorithmic_bytes_per_launch": pr["algorithmic_bytes_per_launch"],
                                      "avg_launch_ms": pr["integrate_avg_launch_ms"]}
    res = {
        "metric": METRIC,
        "value": head_ph["voxel_updates_per_s"],
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head_ph["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large_room_512: one 512^3 volume over 3 m (5.86 mm voxels), 640x480 "
                               "synthetic depth+RGB, 300-frame handheld path, integrate + raycast every frame",
                   "volume_voxels": N_VOX ** 3, "image": [W_IMG, H_IMG], "trunc_voxels": 4, "w_max": 128,
                   "ray_step_voxels": 0.5, "global_batch": 1, "parallelism": "none",
                   "path": "mvf_step (graph)" if head_ph is phases.get("single_step") else "plain calls"},
        "raycast_mpix_s": head_ph["raycast_mpix_s"],
        "integrate_kernel_voxel_updates_per_s": main_ph.get("integrate_kernel_voxel_updates_per_s"),
        "raycast_kernel_mpix_s": main_ph.get("raycast_kernel_mpix_s"),
        "roofline": roof,
        "phases": phases,
    }
    if "tiled" in phases and "batched" in phases:
        res["batched_vs_plain_speedup"] = phases["tiled"]["ms_per_step"] / phases["batched"]["ms_per_step"]
    if "single" in phases and "single_step" in phases:
        res["single_step_vs_plain_speedup"] = phases["single"]["ms_per_step"] / phases["single_step"]["ms_per_step"]
    res["configs"] = config_summary(phases)
    if not args.no_cpu:
        log("cpu baseline (all threads)")
        res["cpu_baseline"] = cpu_baseline(frames, K)
        log("cpu baseline (one thread)")
        one = cpu_baseline(frames, K, budget_s=12.0, threads=1)
        res["cpu_baseline"]["single_thread"] = {k: one[k] for k in
                                                ("value", "integrate_voxel_updates_per_s", "raycast_mpix_s",
                                                 "cores", "sample")}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
