"""CPU oracle for multi-volume TSDF mapping -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP
library in ``paper_1511_07106_amd``; neither imports the other.

The numeric core is plain C (``mvf_oracle.c``, built with gcc
``-O2 -ffp-contract=off``); this module builds it, wraps it with numpy, and
holds the placement policy (plain Python) and the SE(3) exponential used by
finite-difference checks.

Paper: Salvato, Finman, Leonard, arXiv 1511.07106.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mvf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-msse2",
          "-mfpmath=sse", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always, unless ``force`` is False and a
    library newer than the source exists)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def build_variant(defines: Dict[str, int], out_dir: str) -> C.CDLL:
    """Compile the oracle with preprocessor ``defines`` into ``out_dir`` and
    load it.  Only for tests that plant an alternative reading (or a mistake)
    in the oracle to show that a pin rejects it."""
    tag = "_".join(f"{k}{v}" for k, v in sorted(defines.items()))
    path = os.path.join(out_dir, f"liboracle_{tag}.so")
    subprocess.run(["gcc", *CFLAGS, *[f"-D{k}={v}" for k, v in defines.items()], "-o", path, _SRC, "-lm"],
                   check=True)
    return C.CDLL(path)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, np.float32))


# --------------------------------------------------------------------------
# Grid and volumes
# --------------------------------------------------------------------------


@dataclasses.dataclass
class OGrid:
    """World voxel lattice: origin o, voxel size s, truncation in voxels and
    the weight cap.  Global voxel g has its centre at o + s (g + 1/2)."""

    origin: Tuple[float, float, float]
    voxel_size: float
    trunc_voxels: float = 4.0
    w_max: int = 128

    def arr5(self) -> np.ndarray:
        return _f32([*self.origin, self.voxel_size, self.trunc_voxels])

    def arr4(self) -> np.ndarray:
        return _f32([*self.origin, self.voxel_size])

    @property
    def mu(self) -> float:
        return float(np.float32(self.trunc_voxels) * np.float32(self.voxel_size))


@dataclasses.dataclass
class OVolume:
    """Oracle volume state, x-fastest arrays of shape (nz, ny, nx)."""

    dims: Tuple[int, int, int]  # (nx, ny, nz)
    offset: Tuple[int, int, int]  # global voxel offset h_t
    F: np.ndarray  # float64 TSDF (truncation units), 0 where unobserved
    W: np.ndarray  # uint16 weight
    Cc: np.ndarray  # uint8 RGBA (A = colour weight), shape (nz, ny, nx, 4)

    @classmethod
    def empty(cls, dims, offset=(0, 0, 0)) -> "OVolume":
        nx, ny, nz = dims
        return cls(tuple(int(d) for d in dims), tuple(int(o) for o in offset),
                   np.zeros((nz, ny, nx), np.float64), np.zeros((nz, ny, nx), np.uint16),
                   np.zeros((nz, ny, nx, 4), np.uint8))

    def F32(self) -> np.ndarray:
        return self.F.astype(np.float32)


def integrate(vol: OVolume, grid: OGrid, depth: np.ndarray, rgb: Optional[np.ndarray],
              K, T) -> Tuple[int, int, int]:
    """Fuse one frame into ``vol`` in place.  Returns (voxels projecting to a
    valid pixel, voxels updated, voxels in the colour band)."""
    depth = _f32(depth)
    h, w = depth.shape
    rgbc = None if rgb is None else np.ascontiguousarray(rgb, np.uint8)
    if rgbc is not None:
        assert rgbc.shape == (h, w, 3)
    stats = np.zeros(3, np.int64)
    r = lib().orc_integrate(_p(np.asarray(vol.dims, np.int32)), _p(np.asarray(vol.offset, np.int32)),
                            _p(grid.arr5()), C.c_int(grid.w_max), _p(vol.F), _p(vol.W), _p(vol.Cc),
                            _p(depth), _p(rgbc), C.c_int(w), C.c_int(h), _p(_f32(K)),
                            _p(_f32(np.asarray(T).reshape(12))), _p(stats))
    if r != 0:
        raise ValueError("orc_integrate rejected its arguments")
    return int(stats[0]), int(stats[1]), int(stats[2])


def raycast(vols: Sequence[OVolume], grid: OGrid, K, T, width: int, height: int,
            step: float = 0.5, t_far: float = 10.0,
            F32: Optional[Sequence[np.ndarray]] = None, oracle_lib=None) -> Dict[str, np.ndarray]:
    """Raycast one view through all volumes.  ``F32`` optionally gives the
    binary32 TSDF planes to read (default: each volume's F rounded to f32).
    ``oracle_lib``: a variant build from ``build_variant`` (tests only)."""
    n = len(vols)
    if F32 is not None:
        if isinstance(F32, np.ndarray) or len(F32) != n:
            raise TypeError("F32 must be a list with one array per volume")
        for f, v in zip(F32, vols):
            if np.asarray(f).shape != v.W.shape:
                raise ValueError(f"F32 plane of shape {np.asarray(f).shape} for a volume of shape {v.W.shape}")
    dims = np.asarray([v.dims for v in vols], np.int32).reshape(n, 3)
    offs = np.asarray([v.offset for v in vols], np.int32).reshape(n, 3)
    Fs = [(_f32(F32[i]) if F32 is not None else vols[i].F32()).reshape(-1) for i in range(n)]
    Ws = [np.ascontiguousarray(v.W).reshape(-1) for v in vols]
    base = np.zeros(n, np.int64)
    if n > 1:
        base[1:] = np.cumsum([f.size for f in Fs])[:-1]
    Fcat = np.ascontiguousarray(np.concatenate(Fs) if n else np.zeros(1, np.float32))
    Wcat = np.ascontiguousarray(np.concatenate(Ws) if n else np.zeros(1, np.uint16))
    P = width * height
    out = dict(depth=np.zeros(P), vertex=np.zeros((P, 3)), normal=np.zeros((P, 3)),
               hit=np.zeros(P, np.int32), k=np.zeros(P, np.int32), tstar=np.zeros(P, np.float32),
               cells=np.zeros((P, 9), np.int32), ambiguous=np.zeros(P, np.uint8))
    r = (oracle_lib or lib()).orc_raycast(C.c_int(n), _p(dims), _p(offs), _p(Fcat), _p(Wcat), _p(base),
                          _p(grid.arr4()), C.c_float(step), C.c_float(t_far), _p(_f32(K)),
                          _p(_f32(np.asarray(T).reshape(12))), C.c_int(width), C.c_int(height),
                          _p(out["depth"]), _p(out["vertex"]), _p(out["normal"]), _p(out["hit"]),
                          _p(out["k"]), _p(out["tstar"]), _p(out["cells"]), _p(out["ambiguous"]))
    if r != 0:
        raise ValueError("orc_raycast rejected its arguments")
    shp = (height, width)
    return dict(depth=out["depth"].reshape(shp), vertex=out["vertex"].reshape(shp + (3,)),
                normal=out["normal"].reshape(shp + (3,)), hit=out["hit"].reshape(shp),
                k=out["k"].reshape(shp), tstar=out["tstar"].reshape(shp),
                cells=out["cells"].reshape(shp + (9,)), ambiguous=out["ambiguous"].reshape(shp))


def structure(rc: Dict[str, np.ndarray]) -> np.ndarray:
    """Per-pixel frozen structure (k, cell_a, cell_b) from a one-volume raycast
    result, k = -1 where there is no hit."""
    k = rc["k"].reshape(-1, 1)
    cells = rc["cells"].reshape(-1, 9)[:, :6]
    return np.ascontiguousarray(np.concatenate([k, cells], axis=1).astype(np.int32))


def depth_fixed(vol: OVolume, grid: OGrid, K, T64, width, height, kcells,
                step: float = 0.5, F32: Optional[np.ndarray] = None) -> np.ndarray:
    """Binary64 depth at pose ``T64`` with the discrete structure fixed."""
    F = _f32(F32 if F32 is not None else vol.F32())
    out = np.zeros(width * height)
    lib().orc_depth_fixed(_p(np.asarray(vol.dims, np.int32)), _p(np.asarray(vol.offset, np.int32)),
                          _p(F), _p(np.ascontiguousarray(vol.W)), _p(grid.arr4()), C.c_float(step),
                          _p(_f32(K)), _p(np.ascontiguousarray(np.asarray(T64, np.float64).reshape(12))),
                          C.c_int(width), C.c_int(height), _p(np.ascontiguousarray(kcells, np.int32)),
                          _p(out))
    return out.reshape(height, width)


def depth_grad(vol: OVolume, grid: OGrid, K, T64, width, height, kcells, grad_depth,
               step: float = 0.5, F32: Optional[np.ndarray] = None, want_voxels: bool = True):
    """Gradient of sum(grad_depth * depth) w.r.t. the right pose perturbation
    (rho, omega) and the voxel values, binary64."""
    F = _f32(F32 if F32 is not None else vol.F32())
    gxi = np.zeros(6)
    gF = np.zeros(vol.W.shape) if want_voxels else None
    gd = np.ascontiguousarray(np.asarray(grad_depth, np.float64).reshape(-1))
    lib().orc_depth_grad(_p(np.asarray(vol.dims, np.int32)), _p(np.asarray(vol.offset, np.int32)),
                         _p(F), _p(np.ascontiguousarray(vol.W)), _p(grid.arr4()), C.c_float(step),
                         _p(_f32(K)), _p(np.ascontiguousarray(np.asarray(T64, np.float64).reshape(12))),
                         C.c_int(width), C.c_int(height), _p(np.ascontiguousarray(kcells, np.int32)),
                         _p(gd), _p(gxi), _p(gF))
    return gxi, gF


def extract(vol: OVolume, grid: OGrid, F32: Optional[np.ndarray] = None,
            max_points: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Surface points of one volume: at most one vertex per voxel, at the
    linear zero crossing on the first edge (x, y, z) leaving the voxel that
    changes sign inside the truncation band, with the cell's trilinear
    gradient as normal.  ``F32``: the binary32 TSDF to read (default: F
    rounded).  Returns V, N (n x 3, binary64, world) and G (n x 3 global
    voxel), in global voxel order (z, y, x)."""
    F = _f32(F32 if F32 is not None else vol.F32())
    if F.shape != vol.W.shape:
        raise ValueError("F32 must have the volume's shape")
    cap = int(max_points if max_points is not None else max(1, vol.W.size // 4))
    while True:
        V = np.zeros((cap, 3))
        N = np.zeros((cap, 3))
        G = np.zeros((cap, 3), np.int32)
        n = C.c_int64()
        r = lib().orc_extract(_p(np.asarray(vol.dims, np.int32)), _p(np.asarray(vol.offset, np.int32)), _p(F),
                              _p(np.ascontiguousarray(vol.W)), _p(grid.arr4()), C.c_int64(cap), _p(V), _p(N),
                              _p(G), C.byref(n))
        if r != 0:
            raise ValueError("orc_extract rejected its arguments")
        if n.value <= cap or max_points is not None:
            k = min(n.value, cap)
            return dict(V=V[:k], N=N[:k], G=G[:k], n=int(n.value))
        cap = n.value


# --------------------------------------------------------------------------
# SE(3)
# --------------------------------------------------------------------------


def se3_exp(xi) -> np.ndarray:
    """Exp of xi = (rho, omega) as a 3x4 [R | V rho] (binary64)."""
    xi = np.asarray(xi, np.float64)
    rho, w = xi[:3], xi[3:]
    th = float(np.linalg.norm(w))
    Wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-10:
        R = np.eye(3) + Wx + 0.5 * Wx @ Wx
        V = np.eye(3) + 0.5 * Wx + Wx @ Wx / 6.0
    else:
        A = np.sin(th) / th
        B = (1 - np.cos(th)) / th ** 2
        Cc = (th - np.sin(th)) / th ** 3
        R = np.eye(3) + A * Wx + B * Wx @ Wx
        V = np.eye(3) + B * Wx + Cc * Wx @ Wx
    out = np.zeros((3, 4))
    out[:, :3] = R
    out[:, 3] = V @ rho
    return out


def compose(T1, T2) -> np.ndarray:
    T1 = np.asarray(T1, np.float64).reshape(3, 4)
    T2 = np.asarray(T2, np.float64).reshape(3, 4)
    out = np.zeros((3, 4))
    out[:, :3] = T1[:, :3] @ T2[:, :3]
    out[:, 3] = T1[:, :3] @ T2[:, 3] + T1[:, 3]
    return out


# --------------------------------------------------------------------------
# Placement (Dynamic Mapping for SLAM; Insertion and Removal sections)
# --------------------------------------------------------------------------


def placement_counts(depth, K, T, grid: OGrid, d_v: int) -> Dict[Tuple[int, int, int], int]:
    """c(l): number of valid depth rays whose endpoint falls in placement
    cell l (cells of side d_v - 2 voxels)."""
    depth = _f32(depth)
    h, w = depth.shape
    cells = np.zeros((h * w, 3), np.int32)
    valid = np.zeros(h * w, np.uint8)
    r = lib().orc_placement_cells(_p(depth), C.c_int(w), C.c_int(h), _p(_f32(K)),
                                  _p(_f32(np.asarray(T).reshape(12))), _p(grid.arr4()),
                                  C.c_int(d_v), _p(cells), _p(valid))
    if r != 0:
        raise ValueError("orc_placement_cells rejected its arguments")
    keys, cnt = np.unique(cells[valid.astype(bool)], axis=0, return_counts=True)
    return {tuple(int(x) for x in k): int(c) for k, c in zip(keys, cnt)}


def placement_policy(active: Sequence[Tuple[int, int, int]],
                     counts: Dict[Tuple[int, int, int], int], n_max: int,
                     beta: float = 1.5):
    """One insertion/removal step.

    ``active``: cells of the volumes currently in H (unique: a translation
    identifies a volume).  Returns (new active list, added cells, removed
    cells).

    Readings: f fills H up to n_max with the highest-count cells not already
    in H (count descending, then cell lexicographic ascending); afterwards a
    candidate displaces the lowest-count member of H (g removes it) only
    while its count exceeds beta times that member's count.  Members whose
    cell saw no rays this frame count 0; ties among members to remove go to
    the lexicographically larger cell.  Members never displaced stay.
    """
    H = list(dict.fromkeys(tuple(a) for a in active))
    Hs = set(H)
    cand = sorted(((c, k) for k, c in counts.items() if k not in Hs and c > 0),
                  key=lambda ck: (-ck[0], ck[1]))
    added: List[Tuple[int, int, int]] = []
    removed: List[Tuple[int, int, int]] = []
    ci = 0
    while len(H) < n_max and ci < len(cand):
        H.append(cand[ci][1])
        added.append(cand[ci][1])
        ci += 1
    while ci < len(cand) and H:
        c_new, k_new = cand[ci]
        # lowest-count member; ties -> lexicographically larger cell
        low = min(H, key=lambda k: (counts.get(k, 0), tuple(-x for x in k)))
        if c_new > beta * counts.get(low, 0):
            H.remove(low)
            if low in added:
                added.remove(low)
            else:
                removed.append(low)
            H.append(k_new)
            added.append(k_new)
            ci += 1
        else:
            break
    return H, added, removed


def placement_endpoints(depth, K, T, grid: OGrid, d_vs: Sequence[int]):
    """Per valid depth pixel: the global voxel g (int3) holding its ray
    endpoint, and its cell on the placement lattice of each side d_v in
    ``d_vs``.  The voxel is the cell of the side-one lattice (d_v = 3:
    s (d_v - 2) = s), so both come from the same binary32 endpoint formula.
    Returns (g of shape (n, 3), {d_v: cells of shape (n, 3)})."""
    depth = _f32(depth)
    h, w = depth.shape
    out = {}
    ok = np.ones(h * w, bool)
    for d in [3, *d_vs]:
        cells = np.zeros((h * w, 3), np.int32)
        valid = np.zeros(h * w, np.uint8)
        r = lib().orc_placement_cells(_p(depth), C.c_int(w), C.c_int(h), _p(_f32(K)),
                                      _p(_f32(np.asarray(T).reshape(12))), _p(grid.arr4()),
                                      C.c_int(int(d)), _p(cells), _p(valid))
        if r != 0:
            raise ValueError("orc_placement_cells rejected its arguments")
        out[int(d)] = cells
        ok &= valid.astype(bool)
    return out[3][ok], {int(d): out[int(d)][ok] for d in d_vs}


def placement_policy_classes(active: Dict[int, Sequence[Tuple[int, int, int]]], g: np.ndarray,
                             cells: Dict[int, np.ndarray], classes: Sequence[Tuple[int, int]],
                             beta: float = 1.5):
    """One insertion/removal step over volume classes of different sizes on
    one grid (Dynamic Mapping for SLAM: f may choose the volume parameters;
    here the size by count rank).

    ``classes``: (d_v, quota) in rank order, the first class taking the
    highest-count regions.  ``active``: per d_v the cells of its live
    volumes; ``g`` (n, 3): the voxel of each valid ray endpoint; ``cells``:
    per d_v the endpoint cells on that class's lattice (h_t = k (d_v - 2)).

    Classes are taken in order.  Each counts only the endpoints that no live
    volume of an earlier class (as updated this frame) contains, and runs
    the single-size rule of ``placement_policy`` with n_max = its quota.  So
    the largest volumes go where most rays end, the next class covers the
    endpoints they miss, and a volume whose endpoints a larger volume has
    taken over counts 0 and is displaced by the next candidate that beats
    it.  Translations are unique within a class.  Returns ({d_v: new
    active}, {d_v: added}, {d_v: removed})."""
    g = np.asarray(g, np.int64).reshape(-1, 3)
    covered = np.zeros(len(g), bool)
    new_active, added, removed = {}, {}, {}
    for d_v, quota in classes:
        kc = np.asarray(cells[d_v], np.int64).reshape(-1, 3)[~covered]
        # count equal cells: sort them (numpy's lexsort) and measure the runs
        counts: Dict[Tuple[int, int, int], int] = {}
        if len(kc):
            ks = kc[np.lexsort((kc[:, 2], kc[:, 1], kc[:, 0]))]
            starts = np.flatnonzero(np.concatenate([[True], np.any(ks[1:] != ks[:-1], axis=1)]))
            ends = np.concatenate([starts[1:], [len(ks)]])
            counts = {tuple(int(x) for x in ks[a]): int(b - a) for a, b in zip(starts, ends)}
        H, a, r = placement_policy(active.get(d_v, []), counts, quota, beta)
        new_active[d_v], added[d_v], removed[d_v] = H, a, r
        for k in H:
            lo = np.asarray(k, np.int64) * (d_v - 2)
            covered |= np.all((g >= lo) & (g < lo + d_v), axis=1)
    return new_active, added, removed


# --------------------------------------------------------------------------
# Camera tracking (Depth Map Conversion; Camera Tracking: KinectFusion's
# projective point-to-plane ICP)
# --------------------------------------------------------------------------

ICP_LEVELS = 3
ICP_ITERS = (10, 5, 4)        # iterations at levels 0 (full), 1, 2; run coarse to fine
ICP_EPS_D = 0.1               # metres
ICP_COS_THETA = float(np.float32(np.cos(np.radians(20.0))))
ICP_TAU = 0.03                # pyramid: depths within this of the block's first valid one
ICP_SMOOTH = 0.09             # smoothing: neighbours within this of the centre depth (3 x 3 cm)


def level_K(K, level: int) -> np.ndarray:
    """Intrinsics of pyramid level l: f / 2^l, (c + 1/2) / 2^l - 1/2 (binary32)."""
    K = _f32(K)
    sc = np.float32(0.5 ** level)
    h = np.float32(0.5)
    return _f32([K[0] * sc, K[1] * sc, (K[2] + h) * sc - h, (K[3] + h) * sc - h])


def depth_smooth(depth, delta: float = ICP_SMOOTH) -> np.ndarray:
    """Edge-preserving 7x7 binomial smoothing of a depth map (neighbours
    within delta metres of the centre; invalid pixels give 0)."""
    d = _f32(depth)
    h, w = d.shape
    out = np.zeros_like(d)
    lib().orc_depth_smooth(_p(d), C.c_int(w), C.c_int(h), C.c_float(delta), _p(out))
    return out


def depth_pyramid(depth, levels: int = ICP_LEVELS, tau: float = ICP_TAU) -> List[np.ndarray]:
    out = [_f32(depth)]
    for _ in range(1, levels):
        d = out[-1]
        h, w = d.shape
        d2 = np.zeros((h // 2, w // 2), np.float32)
        lib().orc_depth_down(_p(d), C.c_int(w), C.c_int(h), C.c_float(tau), _p(d2))
        out.append(d2)
    return out


def vertex_normal(depth, K) -> Tuple[np.ndarray, np.ndarray]:
    """Vertex and normal maps (h, w, 3) in camera coordinates (NaN: none)."""
    d = _f32(depth)
    h, w = d.shape
    V = np.zeros((h, w, 3), np.float32)
    N = np.zeros((h, w, 3), np.float32)
    lib().orc_vertex_normal(_p(d), C.c_int(w), C.c_int(h), _p(_f32(K)), _p(V), _p(N))
    return V, N


def model_down(V, N) -> Tuple[np.ndarray, np.ndarray]:
    V = _f32(V)
    N = _f32(N)
    h, w = V.shape[:2]
    V2 = np.zeros((h // 2, w // 2, 3), np.float32)
    N2 = np.zeros((h // 2, w // 2, 3), np.float32)
    lib().orc_model_down(_p(V), _p(N), C.c_int(w), C.c_int(h), _p(V2), _p(N2))
    return V2, N2


def icp_reduce(V, N, Vm, Nm, K_level, T, Tm, eps_d: float = ICP_EPS_D, cos_theta: float = ICP_COS_THETA):
    """One association pass: (A 6x6, b 6, inlier count, sum r^2, inlier mask)
    for the estimate T (rounded to binary32 for the decisions)."""
    V, N, Vm, Nm = _f32(V), _f32(N), _f32(Vm), _f32(Nm)
    h, w = V.shape[:2]
    hm, wm = Vm.shape[:2]
    sums = np.zeros(29)
    inl = np.zeros((h, w), np.uint8)
    lib().orc_icp_reduce(_p(V), _p(N), C.c_int(w), C.c_int(h), _p(Vm), _p(Nm), C.c_int(wm), C.c_int(hm),
                         _p(_f32(K_level)), _p(_f32(np.asarray(T).reshape(12))),
                         _p(_f32(np.asarray(Tm).reshape(12))), C.c_float(eps_d), C.c_float(cos_theta),
                         _p(sums), _p(inl))
    A = np.zeros((6, 6))
    k = 0
    for i in range(6):
        for j in range(i, 6):
            A[i, j] = A[j, i] = sums[k]
            k += 1
    return A, sums[21:27].copy(), int(sums[27]), float(sums[28]), inl


def icp_track(depth, K, Vm0, Nm0, Tm, T_init, iters=ICP_ITERS, eps_d: float = ICP_EPS_D,
              cos_theta: float = ICP_COS_THETA, tau: float = ICP_TAU, smooth: float = ICP_SMOOTH):
    """Pose of the frame `depth` against the model maps (Vm0, Nm0: world
    vertex and normal maps rendered at pose Tm, full resolution), from the
    estimate T_init: the depth smoothed (smooth > 0) then its pyramid; levels
    coarse to fine, `iters[l]` Gauss-Newton steps at level l, each solving
    A xi = -b (binary64) and applying T <- Exp(xi) T.  A step with fewer than
    6 pairs, or whose A is not positive definite, leaves T unchanged.
    Returns (T, per-step list of (level, pairs, sum r^2))."""
    levels = len(iters)
    D = depth_pyramid(depth_smooth(depth, smooth) if smooth > 0 else depth, levels, tau)
    Vm, Nm = [_f32(Vm0)], [_f32(Nm0)]
    for _ in range(1, levels):
        v2, n2 = model_down(Vm[-1], Nm[-1])
        Vm.append(v2)
        Nm.append(n2)
    T = np.asarray(T_init, np.float64).reshape(3, 4).copy()
    log = []
    for lvl in reversed(range(levels)):
        Kl = level_K(K, lvl)
        V, N = vertex_normal(D[lvl], Kl)
        for _ in range(iters[lvl]):
            A, b, n, e, _ = icp_reduce(V, N, Vm[lvl], Nm[lvl], Kl, T, Tm, eps_d, cos_theta)
            log.append((lvl, n, e))
            if n < 6:
                continue
            try:
                L = np.linalg.cholesky(A)
            except np.linalg.LinAlgError:
                continue
            xi = -np.linalg.solve(L.T, np.linalg.solve(L, b))
            T = compose(se3_exp(xi), T)
    return T, log
