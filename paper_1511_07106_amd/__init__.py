"""MI355X (gfx950) multi-volume TSDF mapping: the data-parallel core of
Salvato, Finman, Leonard, "Multi-Volume High Resolution RGB-D Mapping with
Dynamic Volume Placement" (arXiv 1511.07106), as hand-written HIP kernels
behind the C ABI in include/mvf.h.  This package is the thin Python binding.
"""
from . import _lib  # noqa: F401
from .api import Context, placement_policy, pose_retract  # noqa: F401

__all__ = ["Context", "placement_policy", "pose_retract"]
