"""MI355X-native information-gain raycasting for Next-Best-Trajectory planning.

The compute path lives in libnbt_ig.so (hand-written HIP for gfx950, C ABI in
include/nbt_ig.h); ``binding`` marshals torch tensors into it.  Importing the
package fails when the library has not been built.
"""

from . import binding
from .binding import (
    NbtError, Context, Map, Batch, Surrogate, CameraT, camera, camera_from_grid, autotune_viewpoints,
    autotune_map, autotune_trajectories, extract_patch, eval_cost, top_k,
    eval_viewpoints, eval_viewpoints_noalloc, eval_trajectories, trace_rays, trace_viewpoints, trace_trajectories, trace_paths, insert_scans, insert_default_params,
    RAY_MISS, RAY_HIT, RAY_END, RAY_EXIT, RAY_INVALID, LAYOUT_LINEAR, LAYOUT_COLUMN4, LAYOUT_COLUMN2, LAYOUT_COLUMN8, LAYOUT_NAMES,
)

__all__ = [
    "binding", "NbtError", "Context", "Map", "Batch", "CameraT", "camera", "camera_from_grid",
    "autotune_viewpoints", "autotune_map", "autotune_trajectories", "Surrogate", "extract_patch", "eval_cost", "top_k",
    "eval_viewpoints", "eval_viewpoints_noalloc", "eval_trajectories", "trace_rays", "trace_viewpoints", "trace_trajectories", "trace_paths", "insert_scans",
    "insert_default_params",
    "RAY_MISS", "RAY_HIT", "RAY_END", "RAY_EXIT", "RAY_INVALID", "LAYOUT_LINEAR", "LAYOUT_COLUMN4", "LAYOUT_COLUMN2", "LAYOUT_COLUMN8", "LAYOUT_NAMES",
]
