"""ctypes declarations of libmvf's C ABI (include/mvf.h).

Loading fails loudly (ImportError) when the HIP library has not been built:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmvf.so")

MVF_OK = 0
MVF_ERR_INVALID_ARG = 1
MVF_ERR_NOT_FOUND = 2
MVF_ERR_OOM = 3
MVF_ERR_BUDGET = 4
MVF_ERR_HIP = 5
MVF_ERR_STATE = 6
MVF_ERR_UNSUPPORTED = 7
MVF_FLAG_TIMING = 1
MVF_EVICT_SWAP_OUT = 1
MVF_AUTOTUNE_OFF = 0
MVF_AUTOTUNE_TUNE = 1
MVF_AUTOTUNE_CACHED = 2


class mvf_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("ray_step", C.c_float), ("t_far", C.c_float),
                ("device", C.c_int32), ("flags", C.c_uint32)]


class mvf_grid_desc(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("voxel_size", C.c_float), ("trunc_voxels", C.c_float),
                ("w_max", C.c_uint16), ("reserved", C.c_uint16)]


class mvf_volume_desc(C.Structure):
    _fields_ = [("grid_id", C.c_int32), ("offset", C.c_int32 * 3), ("dims", C.c_int32 * 3),
                ("stream_id", C.c_int32)]


class mvf_intrinsics(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class mvf_frame(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("rgb", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("depth_pitch", C.c_int32), ("rgb_pitch", C.c_int32)]


class mvf_raycast_out(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("vertex", C.c_void_p), ("normal", C.c_void_p), ("hit", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32)]


class mvf_stats(C.Structure):
    _fields_ = [("voxels_updated", C.c_uint64), ("voxels_band", C.c_uint64), ("pixels_raycast", C.c_uint64),
                ("bytes_h2d", C.c_uint64), ("bytes_d2h", C.c_uint64), ("swaps_in", C.c_uint64),
                ("swaps_out", C.c_uint64), ("integrate_launches", C.c_uint64),
                ("raycast_launches", C.c_uint64), ("step_launches", C.c_uint64),
                ("integrate_ms", C.c_double), ("raycast_ms", C.c_double), ("step_ms", C.c_double),
                ("resident_bytes", C.c_uint64), ("resident_volumes", C.c_int32), ("reserved", C.c_int32),
                ("bricks_projected", C.c_uint64), ("bricks_deep", C.c_uint64)]


class mvf_stream_frame(C.Structure):
    _fields_ = [("stream_id", C.c_int32), ("frame", mvf_frame), ("T_wc", C.c_float * 12),
                ("K", mvf_intrinsics)]


class mvf_schedule(C.Structure):
    _fields_ = [("zchunk", C.c_int32), ("persistent", C.c_int32), ("ray_lanes", C.c_int32),
                ("reserved", C.c_int32)]


class mvf_placement_params(C.Structure):
    _fields_ = [("grid_id", C.c_int32), ("d_v", C.c_int32), ("n_max", C.c_int32), ("beta", C.c_float)]


class mvf_placement_class(C.Structure):
    _fields_ = [("d_v", C.c_int32), ("quota", C.c_int32)]


MVF_MAX_PLACEMENT_CLASSES = 8


class mvf_placement_class_params(C.Structure):
    _fields_ = [("grid_id", C.c_int32), ("n_classes", C.c_int32),
                ("classes", mvf_placement_class * MVF_MAX_PLACEMENT_CLASSES), ("beta", C.c_float),
                ("reserved", C.c_int32)]


class mvf_placement_result(C.Structure):
    _fields_ = [("n_added", C.c_int32), ("n_removed", C.c_int32), ("added", C.c_int32 * 64),
                ("removed", C.c_int32 * 64), ("n_cells", C.c_int32), ("reserved", C.c_int32)]


class mvf_dense_tsdf(C.Structure):
    _fields_ = [("F", C.c_void_p), ("W", C.c_void_p), ("dims", C.c_int32 * 3), ("offset", C.c_int32 * 3),
                ("origin", C.c_float * 3), ("voxel_size", C.c_float), ("generation", C.c_uint64)]


class mvf_track_model(C.Structure):
    _fields_ = [("vertex", C.c_void_p), ("normal", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("T_wc", C.c_float * 12)]


class mvf_track_params(C.Structure):
    _fields_ = [("levels", C.c_int32), ("iters", C.c_int32 * 3), ("eps_d", C.c_float), ("cos_theta", C.c_float),
                ("tau", C.c_float), ("smooth", C.c_float)]


class mvf_track_stats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("pairs", C.c_int32 * 64), ("sq_err", C.c_double * 64)]


P = C.c_void_p
I32 = C.c_int32
PI32 = C.POINTER(C.c_int32)
PF = C.POINTER(C.c_float)
PD = C.POINTER(C.c_double)

# user-defined placement function (mvf_placement_fn)
PLACEMENT_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_int32, C.c_int32, PI32, C.c_int32, PI32, PI32, C.c_int32,
                           C.c_int32, PI32, PI32)

# name -> (argtypes); every function returns mvf_status (int32) unless listed
SIGNATURES = {
    "mvf_create": [C.POINTER(P), C.POINTER(mvf_config)],
    "mvf_destroy": [P],
    "mvf_synchronize": [P],
    "mvf_set_budget": [P, C.c_uint64],
    "mvf_get_stats": [P, C.POINTER(mvf_stats)],
    "mvf_reset_stats": [P],
    "mvf_grid_create": [P, C.POINTER(mvf_grid_desc), PI32],
    "mvf_volume_create": [P, C.POINTER(mvf_volume_desc), PI32],
    "mvf_volume_destroy": [P, I32],
    "mvf_volume_place": [P, I32],
    "mvf_volume_evict": [P, I32, C.c_uint32],
    "mvf_volume_swap_in": [P, I32, P],
    "mvf_volume_swap_out": [P, I32, P],
    "mvf_volume_read": [P, I32, P, P, P],
    "mvf_volume_brick_summary": [P, I32, P, P],
    "mvf_volume_write": [P, I32, P, P, P],
    "mvf_volume_query": [P, I32, PI32, C.POINTER(C.c_uint64), PI32],
    "mvf_volume_describe": [P, I32, C.POINTER(mvf_volume_desc)],
    "mvf_volume_extract": [P, I32, P, P, P, C.c_int64, C.POINTER(C.c_int64), P],
    "mvf_integrate": [P, I32, C.POINTER(mvf_frame), PF, C.POINTER(mvf_intrinsics), P],
    "mvf_raycast": [P, I32, PF, C.POINTER(mvf_intrinsics), C.POINTER(mvf_raycast_out), P],
    "mvf_step": [P, I32, C.POINTER(mvf_stream_frame), C.POINTER(mvf_raycast_out), P],
    "mvf_set_schedule": [P, C.POINTER(mvf_schedule)],
    "mvf_get_schedule": [P, C.POINTER(mvf_schedule)],
    "mvf_autotune": [P, I32, C.c_char_p],
    "mvf_placement_update": [P, I32, C.POINTER(mvf_frame), PF, C.POINTER(mvf_intrinsics),
                             C.POINTER(mvf_placement_params), C.POINTER(mvf_placement_result), P],
    "mvf_placement_update_classes": [P, I32, C.POINTER(mvf_frame), PF, C.POINTER(mvf_intrinsics),
                                     C.POINTER(mvf_placement_class_params), C.POINTER(mvf_placement_result), P],
    "mvf_placement_update_custom": [P, I32, C.POINTER(mvf_frame), PF, C.POINTER(mvf_intrinsics),
                                    C.POINTER(mvf_placement_class_params), PLACEMENT_FN, P,
                                    C.POINTER(mvf_placement_result), P],
    "mvf_placement_count": [P, C.POINTER(mvf_frame), PF, C.POINTER(mvf_intrinsics), I32, I32, PI32, PI32,
                            I32, PI32, P],
    "mvf_placement_policy": [PI32, I32, PI32, PI32, I32, I32, C.c_float, PI32, PI32, PI32, PI32, PI32, PI32],
    "mvf_diffray_forward": [P, C.POINTER(mvf_dense_tsdf), PF, C.POINTER(mvf_intrinsics), I32, I32, P, P, P],
    "mvf_diffray_backward": [P, C.POINTER(mvf_dense_tsdf), PF, C.POINTER(mvf_intrinsics), I32, I32, P, P, P,
                             P, P],
    "mvf_diffray_backward_noalloc": [P, C.POINTER(mvf_dense_tsdf), PF, C.POINTER(mvf_intrinsics), I32, I32, P, P,
                                     P, P, P],
    "mvf_depth_maps": [P, C.POINTER(mvf_frame), C.POINTER(mvf_intrinsics), I32, C.c_float, C.c_float, P, P, P],
    "mvf_track": [P, C.POINTER(mvf_frame), C.POINTER(mvf_intrinsics), C.POINTER(mvf_track_model), PD,
                  C.POINTER(mvf_track_params), PD, C.POINTER(mvf_track_stats), P],
    "mvf_checkpoint_save": [P, C.c_char_p],
    "mvf_checkpoint_load": [P, C.c_char_p],
    "mvf_pose_retract": [PD, PD, PD],
    "mvf_pose_right_jacobian": [PD, PD],
}
STRING_FUNCS = {"mvf_status_string": [I32], "mvf_last_error": [], "mvf_version": []}

_lib = None


def load() -> C.CDLL:
    """Load libmvf.so and declare its functions.  Raises ImportError if the
    library is missing (run paper_1511_07106_amd.build first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmvf.so not built at {LIB_PATH}; run `python -m paper_1511_07106_amd.build`")
    # torch ships its own HIP runtime under the same soname; importing torch
    # first makes libmvf bind to that one, so the process holds a single HIP
    # runtime (the reverse order leaves torch on a runtime it was not built
    # against, and it then finds no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int32
    for name, args in STRING_FUNCS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_char_p
    _lib = lib
    return lib


class MvfError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        super().__init__(f"{func}: {message} (status {status})")
        self.status = status


def check(status: int, func: str) -> None:
    if status != MVF_OK:
        lib = load()
        raise MvfError(status, func, lib.mvf_last_error().decode(errors="replace"))


def exported_names():
    return list(SIGNATURES) + list(STRING_FUNCS)
