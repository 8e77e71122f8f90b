"""Python binding of libmvf: argument marshalling only.

Every step of the mapping path runs in the HIP library; PyTorch provides
device memory (tensors) and the stream (torch's current HIP stream).
Poses are 3x4 camera-to-world [R | t] (OpenCV axes), intrinsics
(fx, fy, cx, cy).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _stream(stream=None) -> C.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(int(s.cuda_stream))


def _pose(T) -> C.Array:
    a = np.asarray(T, dtype=np.float64).reshape(-1)
    if a.size != 12:
        raise ValueError("pose must be 3x4")
    return (C.c_float * 12)(*[float(np.float32(x)) for x in a])


def _K(K) -> L.mvf_intrinsics:
    k = [float(np.float32(x)) for x in np.asarray(K, dtype=np.float64).reshape(-1)[:4]]
    return L.mvf_intrinsics(*k)


def _dev_ptr(t, dtype, shape_tail=None, name="tensor"):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a HIP device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[-len(shape_tail):]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


class Context:
    """One mapping context on one HIP device (owns volumes and their memory)."""

    def __init__(self, budget_bytes: int = 0, ray_step: float = 0.5, t_far: float = 10.0,
                 device: int = 0, timing: bool = False):
        self.lib = L.load()
        cfg = L.mvf_config(int(budget_bytes), float(ray_step), float(t_far), int(device),
                           L.MVF_FLAG_TIMING if timing else 0)
        h = C.c_void_p()
        L.check(self.lib.mvf_create(C.byref(h), C.byref(cfg)), "mvf_create")
        self.h = h
        self.device = device
        self._grids: Dict[int, L.mvf_grid_desc] = {}
        self._vols: Dict[int, L.mvf_volume_desc] = {}

    # -- lifetime ---------------------------------------------------------
    def close(self) -> None:
        if self.h:
            L.check(self.lib.mvf_destroy(self.h), "mvf_destroy")
            self.h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.mvf_destroy(self.h)
        except Exception:
            pass

    def synchronize(self) -> None:
        L.check(self.lib.mvf_synchronize(self.h), "mvf_synchronize")

    def set_budget(self, nbytes: int) -> None:
        L.check(self.lib.mvf_set_budget(self.h, C.c_uint64(int(nbytes))), "mvf_set_budget")

    def stats(self) -> Dict[str, float]:
        s = L.mvf_stats()
        L.check(self.lib.mvf_get_stats(self.h, C.byref(s)), "mvf_get_stats")
        return {f: getattr(s, f) for f, _ in L.mvf_stats._fields_ if f != "reserved"}

    def reset_stats(self) -> None:
        L.check(self.lib.mvf_reset_stats(self.h), "mvf_reset_stats")

    # -- grids and volumes ----------------------------------------------
    def grid(self, origin, voxel_size: float, trunc_voxels: float = 4.0, w_max: int = 128) -> int:
        d = L.mvf_grid_desc((C.c_float * 3)(*[float(x) for x in origin]), float(voxel_size),
                            float(trunc_voxels), int(w_max), 0)
        gid = C.c_int32()
        L.check(self.lib.mvf_grid_create(self.h, C.byref(d), C.byref(gid)), "mvf_grid_create")
        self._grids[gid.value] = d
        return gid.value

    def volume(self, grid_id: int, offset, dims, stream_id: int = 0, place: bool = True) -> int:
        d = L.mvf_volume_desc(int(grid_id), (C.c_int32 * 3)(*[int(x) for x in offset]),
                              (C.c_int32 * 3)(*[int(x) for x in dims]), int(stream_id))
        vid = C.c_int32()
        L.check(self.lib.mvf_volume_create(self.h, C.byref(d), C.byref(vid)), "mvf_volume_create")
        self._vols[vid.value] = d
        if place:
            self.place(vid.value)
        return vid.value

    def destroy_volume(self, vid: int) -> None:
        L.check(self.lib.mvf_volume_destroy(self.h, int(vid)), "mvf_volume_destroy")
        self._vols.pop(vid, None)

    def place(self, vid: int) -> None:
        L.check(self.lib.mvf_volume_place(self.h, int(vid)), "mvf_volume_place")

    def evict(self, vid: int, swap_out: bool = False) -> None:
        L.check(self.lib.mvf_volume_evict(self.h, int(vid), L.MVF_EVICT_SWAP_OUT if swap_out else 0),
                "mvf_volume_evict")

    def swap_in(self, vid: int, stream=None) -> None:
        L.check(self.lib.mvf_volume_swap_in(self.h, int(vid), _stream(stream)), "mvf_volume_swap_in")

    def swap_out(self, vid: int, stream=None) -> None:
        L.check(self.lib.mvf_volume_swap_out(self.h, int(vid), _stream(stream)), "mvf_volume_swap_out")

    def query(self, vid: int) -> Tuple[bool, int, bool]:
        r, b, a = C.c_int32(), C.c_uint64(), C.c_int32()
        L.check(self.lib.mvf_volume_query(self.h, int(vid), C.byref(r), C.byref(b), C.byref(a)),
                "mvf_volume_query")
        return bool(r.value), int(b.value), bool(a.value)

    def describe(self, vid: int) -> L.mvf_volume_desc:
        d = L.mvf_volume_desc()
        L.check(self.lib.mvf_volume_describe(self.h, int(vid), C.byref(d)), "mvf_volume_describe")
        return d

    def dims(self, vid: int) -> Tuple[int, int, int]:
        return tuple(self.describe(vid).dims)

    def offset(self, vid: int) -> Tuple[int, int, int]:
        return tuple(self.describe(vid).offset)

    def read_volume(self, vid: int):
        """(F float32, W uint16, RGBA uint8) arrays of shape (nz, ny, nx[, 4])."""
        nx, ny, nz = self.dims(vid)
        F = np.zeros((nz, ny, nx), np.float32)
        W = np.zeros((nz, ny, nx), np.uint16)
        Cc = np.zeros((nz, ny, nx, 4), np.uint8)
        L.check(self.lib.mvf_volume_read(self.h, int(vid), F.ctypes.data_as(C.c_void_p),
                                         W.ctypes.data_as(C.c_void_p), Cc.ctypes.data_as(C.c_void_p)),
                "mvf_volume_read")
        return F, W, Cc

    def brick_summary(self, vid: int):
        """(flag, dist) uint8 arrays of shape (bx, by, bz) = ceil(dims / 8):
        the raycast's exact-skip flags and capped Chebyshev distances."""
        nb = [(d + 7) // 8 for d in self.dims(vid)]
        flag = np.zeros(nb, np.uint8)
        dist = np.zeros(nb, np.uint8)
        L.check(self.lib.mvf_volume_brick_summary(self.h, int(vid), flag.ctypes.data_as(C.c_void_p),
                                                  dist.ctypes.data_as(C.c_void_p)), "mvf_volume_brick_summary")
        return flag, dist

    def extract(self, vid: int, with_index: bool = True, stream=None):
        """Surface points of a volume on the device: dict of V, N ((n, 3)
        float32 tensors, world metres and unit normals) and G ((n, 3) int32
        global voxel indices, if with_index), in the library's brick order.
        Counts first, then allocates exactly and emits."""
        torch = _torch()
        n = C.c_int64()
        L.check(self.lib.mvf_volume_extract(self.h, int(vid), None, None, None, 0, C.byref(n), _stream(stream)),
                "mvf_volume_extract")
        dev = torch.device("cuda", self.device)
        k = int(n.value)
        V = torch.empty((k, 3), dtype=torch.float32, device=dev)
        N = torch.empty((k, 3), dtype=torch.float32, device=dev)
        G = torch.empty((k, 3), dtype=torch.int32, device=dev) if with_index else None
        if k:
            L.check(self.lib.mvf_volume_extract(self.h, int(vid), C.c_void_p(V.data_ptr()),
                                                C.c_void_p(N.data_ptr()),
                                                C.c_void_p(G.data_ptr()) if G is not None else None,
                                                k, C.byref(n), _stream(stream)), "mvf_volume_extract")
        out = {"V": V, "N": N, "n": k}
        if G is not None:
            out["G"] = G
        return out

    def export_points(self, vids, with_index: bool = False):
        """The surface points of each volume in vids (for instance the ids a
        placement update removed: the paper downloads a removed volume's
        point cloud), as {id: extract(id)}."""
        return {int(v): self.extract(int(v), with_index=with_index) for v in vids}

    def save(self, path: str) -> None:
        """Checkpoint the context (grids, volumes and their state, placement
        bookkeeping) to `path`."""
        L.check(self.lib.mvf_checkpoint_save(self.h, os.fsencode(path)), "mvf_checkpoint_save")

    def load(self, path: str) -> None:
        """Restore a checkpoint into this (empty) context."""
        L.check(self.lib.mvf_checkpoint_load(self.h, os.fsencode(path)), "mvf_checkpoint_load")

    def write_volume(self, vid: int, F=None, W=None, rgba=None) -> None:
        nx, ny, nz = self.dims(vid)
        arrs = []
        for a, dt, shp in ((F, np.float32, (nz, ny, nx)), (W, np.uint16, (nz, ny, nx)),
                           (rgba, np.uint8, (nz, ny, nx, 4))):
            if a is None:
                arrs.append(None)
                continue
            a = np.ascontiguousarray(a, dtype=dt)
            if a.shape != shp:
                raise ValueError(f"expected shape {shp}, got {a.shape}")
            arrs.append(a)
        ptrs = [None if a is None else a.ctypes.data_as(C.c_void_p) for a in arrs]
        L.check(self.lib.mvf_volume_write(self.h, int(vid), *ptrs), "mvf_volume_write")

    # -- per-frame path ----------------------------------------------------
    @staticmethod
    def _frame(depth, rgb) -> L.mvf_frame:
        torch = _torch()
        if depth.dim() != 2:
            raise ValueError("depth must be (H, W)")
        H, W = depth.shape
        dp = _dev_ptr(depth, torch.float32, name="depth")
        rp = _dev_ptr(rgb, torch.uint8, (H, W, 3), name="rgb") if rgb is not None else None
        return L.mvf_frame(dp, rp, W, H, 0, 0)

    def integrate(self, depth, rgb, T, K, stream_id: int = 0, stream=None) -> None:
        f = self._frame(depth, rgb)
        L.check(self.lib.mvf_integrate(self.h, int(stream_id), C.byref(f), _pose(T), C.byref(_K(K)),
                                       _stream(stream)), "mvf_integrate")

    def raycast(self, T, K, width: int, height: int, stream_id: int = 0, out=None, stream=None,
                want_vertex: bool = True, want_normal: bool = True, want_hit: bool = True):
        torch = _torch()
        dev = torch.device("cuda", self.device)
        if out is None:
            out = {"depth": torch.empty((height, width), dtype=torch.float32, device=dev)}
            if want_vertex:
                out["vertex"] = torch.empty((height, width, 3), dtype=torch.float32, device=dev)
            if want_normal:
                out["normal"] = torch.empty((height, width, 3), dtype=torch.float32, device=dev)
            if want_hit:
                out["hit"] = torch.empty((height, width), dtype=torch.int32, device=dev)
        o = self._out_struct(out, width, height)
        L.check(self.lib.mvf_raycast(self.h, int(stream_id), _pose(T), C.byref(_K(K)), C.byref(o),
                                     _stream(stream)), "mvf_raycast")
        return out

    @staticmethod
    def _out_struct(out, width, height) -> L.mvf_raycast_out:
        torch = _torch()
        return L.mvf_raycast_out(_dev_ptr(out["depth"], torch.float32, (height, width), "depth"),
                                 _dev_ptr(out.get("vertex"), torch.float32, (height, width, 3), "vertex"),
                                 _dev_ptr(out.get("normal"), torch.float32, (height, width, 3), "normal"),
                                 _dev_ptr(out.get("hit"), torch.int32, (height, width), "hit"),
                                 width, height)

    def step(self, frames: Sequence[Tuple[int, object, object, object, object]], outs: Sequence[dict],
             stream=None) -> None:
        """Batched form: frames = [(stream_id, depth, rgb, T, K)], outs = raycast
        output dicts (same keys as raycast())."""
        n = len(frames)
        arr = (L.mvf_stream_frame * n)()
        oarr = (L.mvf_raycast_out * n)()
        for i, (sid, depth, rgb, T, K) in enumerate(frames):
            arr[i].stream_id = int(sid)
            arr[i].frame = self._frame(depth, rgb)
            arr[i].T_wc = _pose(T)
            arr[i].K = _K(K)
            h, w = outs[i]["depth"].shape
            oarr[i] = self._out_struct(outs[i], w, h)
        L.check(self.lib.mvf_step(self.h, n, arr, oarr, _stream(stream)), "mvf_step")

    def set_schedule(self, zchunk: int = 4, persistent: int = 0, ray_lanes: int = 4) -> None:
        """Fix the launch schedule of step() (switches autotuning off)."""
        sc = L.mvf_schedule(int(zchunk), int(persistent), int(ray_lanes), 0)
        L.check(self.lib.mvf_set_schedule(self.h, C.byref(sc)), "mvf_set_schedule")

    def schedule(self) -> Dict[str, int]:
        """The schedule the last step() ran with."""
        sc = L.mvf_schedule()
        L.check(self.lib.mvf_get_schedule(self.h, C.byref(sc)), "mvf_get_schedule")
        return {"zchunk": sc.zchunk, "persistent": sc.persistent, "ray_lanes": sc.ray_lanes}

    def autotune(self, mode: str = "tune", cache_path: Optional[str] = None) -> None:
        """mode: 'off', 'tune' (time the candidate schedules on the first
        steps of each new shape) or 'cached' (use cache_path only)."""
        m = {"off": L.MVF_AUTOTUNE_OFF, "tune": L.MVF_AUTOTUNE_TUNE, "cached": L.MVF_AUTOTUNE_CACHED}[mode]
        path = cache_path.encode() if cache_path else None
        L.check(self.lib.mvf_autotune(self.h, m, path), "mvf_autotune")

    # -- placement -----------------------------------------------------------
    def placement_count(self, depth, T, K, grid_id: int, d_v: int, max_cells: int = 8192, stream=None):
        f = self._frame(depth, None)
        cells = np.zeros((max_cells, 3), np.int32)
        counts = np.zeros(max_cells, np.int32)
        n = C.c_int32()
        L.check(self.lib.mvf_placement_count(self.h, C.byref(f), _pose(T), C.byref(_K(K)), int(grid_id),
                                             int(d_v), cells.ctypes.data_as(L.PI32),
                                             counts.ctypes.data_as(L.PI32), max_cells, C.byref(n),
                                             _stream(stream)), "mvf_placement_count")
        k = min(n.value, max_cells)
        return {tuple(int(x) for x in cells[i]): int(counts[i]) for i in range(k)}

    def placement_update(self, depth, T, K, grid_id: int, d_v: int, n_max: int, beta: float = 1.5,
                         stream_id: int = 0, stream=None):
        f = self._frame(depth, None)
        p = L.mvf_placement_params(int(grid_id), int(d_v), int(n_max), float(beta))
        r = L.mvf_placement_result()
        L.check(self.lib.mvf_placement_update(self.h, int(stream_id), C.byref(f), _pose(T), C.byref(_K(K)),
                                              C.byref(p), C.byref(r), _stream(stream)),
                "mvf_placement_update")
        return list(r.added[:r.n_added]), list(r.removed[:r.n_removed]), r.n_cells

    def placement_update_classes(self, depth, T, K, grid_id: int, classes, beta: float = 1.5,
                                 stream_id: int = 0, stream=None):
        """Placement with volumes of several sizes: ``classes`` is a list of
        (d_v, quota) in rank order (the first class takes the highest-count
        regions).  Returns (added ids, removed ids, distinct cells)."""
        f = self._frame(depth, None)
        p = L.mvf_placement_class_params()
        p.grid_id = int(grid_id)
        p.n_classes = len(classes)
        if not 1 <= len(classes) <= L.MVF_MAX_PLACEMENT_CLASSES:
            raise ValueError(f"between 1 and {L.MVF_MAX_PLACEMENT_CLASSES} classes")
        for i, (d_v, quota) in enumerate(classes):
            p.classes[i].d_v = int(d_v)
            p.classes[i].quota = int(quota)
        p.beta = float(beta)
        r = L.mvf_placement_result()
        L.check(self.lib.mvf_placement_update_classes(self.h, int(stream_id), C.byref(f), _pose(T),
                                                      C.byref(_K(K)), C.byref(p), C.byref(r), _stream(stream)),
                "mvf_placement_update_classes")
        return list(r.added[:r.n_added]), list(r.removed[:r.n_removed]), r.n_cells

    def placement_update_custom(self, depth, T, K, grid_id: int, classes, policy, stream_id: int = 0,
                                stream=None):
        """Placement with a user-defined insertion f.  ``classes``: (d_v,
        quota) in rank order.  ``policy(class_index, d_v, live, counts,
        quota)`` gets the class's live cells (list of 3-tuples) and this
        frame's endpoint counts ({cell: count}, counted on the device) and
        returns the class's live cells after the update (at most quota).
        Returns (added ids, removed ids, distinct cells)."""
        f = self._frame(depth, None)
        p = L.mvf_placement_class_params()
        p.grid_id = int(grid_id)
        if not 1 <= len(classes) <= L.MVF_MAX_PLACEMENT_CLASSES:
            raise ValueError(f"between 1 and {L.MVF_MAX_PLACEMENT_CLASSES} classes")
        p.n_classes = len(classes)
        for i, (d_v, quota) in enumerate(classes):
            p.classes[i].d_v = int(d_v)
            p.classes[i].quota = int(quota)
        p.beta = 1.0
        failure = []

        def trampoline(_user, ci, d_v, live, n_live, cells, counts, n_cells, quota, keep, n_keep):
            try:
                lv = [(live[3 * i], live[3 * i + 1], live[3 * i + 2]) for i in range(n_live)]
                cnt = {(cells[3 * i], cells[3 * i + 1], cells[3 * i + 2]): counts[i] for i in range(n_cells)}
                out = [tuple(int(x) for x in k) for k in policy(int(ci), int(d_v), lv, cnt, int(quota))]
                if len(out) > quota:
                    raise ValueError(f"policy kept {len(out)} cells, quota {quota}")
                for i, k in enumerate(out):
                    keep[3 * i], keep[3 * i + 1], keep[3 * i + 2] = k
                n_keep[0] = len(out)
                return 0
            except BaseException as e:  # noqa: BLE001 -- re-raised after the C call returns
                failure.append(e)
                return 1

        cb = L.PLACEMENT_FN(trampoline)
        r = L.mvf_placement_result()
        st = self.lib.mvf_placement_update_custom(self.h, int(stream_id), C.byref(f), _pose(T), C.byref(_K(K)),
                                                  C.byref(p), cb, None, C.byref(r), _stream(stream))
        if failure:
            raise failure[0]
        L.check(st, "mvf_placement_update_custom")
        return list(r.added[:r.n_added]), list(r.removed[:r.n_removed]), r.n_cells

    # -- camera tracking ------------------------------------------------------
    def depth_maps(self, depth, K, level: int = 0, tau: float = 0.03, smooth: float = 0.09, stream=None):
        """Vertex and normal maps ((h >> level, w >> level, 3) float32 tensors,
        camera frame, NaN where undefined) of a depth frame's pyramid level
        (after the edge-preserving smoothing when smooth > 0)."""
        torch = _torch()
        f = self._frame(depth, None)
        H, W = depth.shape
        dev = depth.device
        V = torch.empty((H >> level, W >> level, 3), dtype=torch.float32, device=dev)
        N = torch.empty_like(V)
        L.check(self.lib.mvf_depth_maps(self.h, C.byref(f), C.byref(_K(K)), int(level), float(tau), float(smooth),
                                        C.c_void_p(V.data_ptr()), C.c_void_p(N.data_ptr()), _stream(stream)),
                "mvf_depth_maps")
        return V, N

    def track(self, depth, K, model, T_model, T_init, iters=(10, 5, 4), eps_d: float = 0.1,
              cos_theta: float = 0.9396926164627075, tau: float = 0.03, smooth: float = 0.09, stream=None):
        """Pose of `depth` by projective point-to-plane ICP against `model`
        (a dict with the previous raycast's "vertex" and "normal" maps, world
        frame, rendered at T_model), from T_init.  iters: Gauss-Newton steps
        at levels 0, 1, 2 (its length sets the pyramid depth).  Returns
        (T (3, 4) float64, {"pairs": [...], "sq_err": [...]} per step)."""
        torch = _torch()
        f = self._frame(depth, None)
        H, W = depth.shape
        m = L.mvf_track_model()
        m.vertex = _dev_ptr(model["vertex"], torch.float32, (H, W, 3), "model vertex")
        m.normal = _dev_ptr(model["normal"], torch.float32, (H, W, 3), "model normal")
        m.width, m.height = W, H
        m.T_wc = _pose(T_model)
        p = L.mvf_track_params()
        p.levels = len(iters)
        for i, n in enumerate(iters):
            p.iters[i] = int(n)
        p.eps_d, p.cos_theta, p.tau, p.smooth = float(eps_d), float(cos_theta), float(tau), float(smooth)
        Ti = np.ascontiguousarray(np.asarray(T_init, np.float64).reshape(12))
        To = np.zeros(12)
        st = L.mvf_track_stats()
        L.check(self.lib.mvf_track(self.h, C.byref(f), C.byref(_K(K)), C.byref(m), Ti.ctypes.data_as(L.PD),
                                   C.byref(p), To.ctypes.data_as(L.PD), C.byref(st), _stream(stream)), "mvf_track")
        return To.reshape(3, 4), {"pairs": list(st.pairs[:st.steps]), "sq_err": list(st.sq_err[:st.steps])}

    # -- differentiable raycast ------------------------------------------------
    @staticmethod
    def _dense(F, W, origin, voxel_size, offset=(0, 0, 0), generation: int = 0) -> L.mvf_dense_tsdf:
        torch = _torch()
        if F.dim() != 3 or W.shape != F.shape:
            raise ValueError("F and W must be (nz, ny, nx) of equal shape")
        nz, ny, nx = F.shape
        return L.mvf_dense_tsdf(_dev_ptr(F, torch.float32, name="F"), _dev_ptr(W, torch.int16, name="W")
                                if W.dtype == torch.int16 else _dev_ptr(W, torch.uint16, name="W"),
                                (C.c_int32 * 3)(nx, ny, nz), (C.c_int32 * 3)(*[int(x) for x in offset]),
                                (C.c_float * 3)(*[float(x) for x in origin]), float(voxel_size), int(generation))

    def diffray_forward(self, F, W, origin, voxel_size, T, K, width, height, offset=(0, 0, 0),
                        stream=None, generation: int = 0):
        """Depth (H, W) float32 and crossing record (H, W) int32.  generation:
        0 rebuilds the library's copy of (F, W) on this call; a non-zero value
        reuses the copy built by the last call with the same tensors and
        generation (bump it after changing F or W)."""
        torch = _torch()
        dev = F.device
        depth = torch.empty((height, width), dtype=torch.float32, device=dev)
        record = torch.empty((height, width), dtype=torch.int32, device=dev)
        v = self._dense(F, W, origin, voxel_size, offset, generation)
        L.check(self.lib.mvf_diffray_forward(self.h, C.byref(v), _pose(T), C.byref(_K(K)), int(width),
                                             int(height), C.c_void_p(depth.data_ptr()),
                                             C.c_void_p(record.data_ptr()), _stream(stream)),
                "mvf_diffray_forward")
        return depth, record

    def diffray_backward(self, F, W, origin, voxel_size, T, K, grad_depth, record, grad_F=None,
                         offset=(0, 0, 0), stream=None, grad_xi=None, noalloc=False):
        """dL/dxi (6 doubles on the device; written into ``grad_xi`` when
        given) and dL/dF accumulated into ``grad_F``.  ``noalloc`` calls
        mvf_diffray_backward_noalloc, which allocates no device memory."""
        torch = _torch()
        h, w = record.shape
        gxi = torch.zeros(6, dtype=torch.float64, device=F.device) if grad_xi is None else grad_xi
        v = self._dense(F, W, origin, voxel_size, offset)
        gd = grad_depth.contiguous()
        name = "mvf_diffray_backward_noalloc" if noalloc else "mvf_diffray_backward"
        L.check(getattr(self.lib, name)(
            self.h, C.byref(v), _pose(T), C.byref(_K(K)), int(w), int(h),
            _dev_ptr(gd, torch.float32, (h, w), "grad_depth"), _dev_ptr(record, torch.int32, (h, w), "record"),
            _dev_ptr(grad_F, torch.float32, name="grad_F") if grad_F is not None else None,
            _dev_ptr(gxi, torch.float64, (6,), "grad_xi"), _stream(stream)), name)
        return gxi


def placement_policy(active, counts: Dict[Tuple[int, int, int], int], n_max: int, beta: float = 1.5):
    """Host-only insertion/removal step of the C library on cell keys."""
    lib = L.load()
    act = np.ascontiguousarray(np.asarray(list(active), np.int32).reshape(-1, 3))
    keys = list(counts.keys())
    cells = np.ascontiguousarray(np.asarray(keys, np.int32).reshape(-1, 3))
    cnt = np.ascontiguousarray(np.asarray([counts[k] for k in keys], np.int32))
    cap = len(act) + len(keys) + 1
    out = np.zeros((max(n_max, 1), 3), np.int32)
    add = np.zeros((cap, 3), np.int32)
    rem = np.zeros((cap, 3), np.int32)
    n_out, n_add, n_rem = C.c_int32(), C.c_int32(), C.c_int32()
    L.check(lib.mvf_placement_policy(act.ctypes.data_as(L.PI32), len(act), cells.ctypes.data_as(L.PI32),
                                     cnt.ctypes.data_as(L.PI32), len(keys), int(n_max), float(beta),
                                     out.ctypes.data_as(L.PI32), C.byref(n_out), add.ctypes.data_as(L.PI32),
                                     C.byref(n_add), rem.ctypes.data_as(L.PI32), C.byref(n_rem)),
            "mvf_placement_policy")
    tup = lambda a, n: [tuple(int(x) for x in a[i]) for i in range(n)]
    return tup(out, n_out.value), tup(add, n_add.value), tup(rem, n_rem.value)


def pose_retract(T, xi) -> np.ndarray:
    lib = L.load()
    Ta = np.ascontiguousarray(np.asarray(T, np.float64).reshape(12))
    xa = np.ascontiguousarray(np.asarray(xi, np.float64).reshape(6))
    out = np.zeros(12)
    L.check(lib.mvf_pose_retract(Ta.ctypes.data_as(L.PD), xa.ctypes.data_as(L.PD), out.ctypes.data_as(L.PD)),
            "mvf_pose_retract")
    return out.reshape(3, 4)


def pose_right_jacobian(xi) -> np.ndarray:
    """J (6x6) with T Exp(xi + d) = T Exp(xi) Exp(J d) to first order."""
    lib = L.load()
    xa = np.ascontiguousarray(np.asarray(xi, np.float64).reshape(6))
    out = np.zeros(36)
    L.check(lib.mvf_pose_right_jacobian(xa.ctypes.data_as(L.PD), out.ctypes.data_as(L.PD)),
            "mvf_pose_right_jacobian")
    return out.reshape(6, 6)
