"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package only draws random scenes, camera poses and trajectories with
NumPy's PCG64 generator.  It holds none of the information-gain arithmetic
(no voxel gains, no ray traversal, no reductions): both the oracle and the
GPU library consume the float32 arrays produced here, so parity does not
depend on any choice made in this package.

Seeds follow one rule everywhere: ``seed = 22588 + 1000 * cfg + map_idx``
for scenes and ``scene_seed + 500`` for the poses drawn in that scene.
"""

from .scenes import (
    SceneMap,
    scene_spheres,
    scene_tabletop,
    scene_uniform,
    batch_maps,
)
from .poses import (
    look_at,
    poses_sphere,
    poses_shell,
    poses_ball,
    trajectories_walk,
)
from .configs import (
    Camera,
    Workload,
    make_config,
    scene_seed,
    pose_seed,
)

__all__ = [
    "SceneMap", "scene_spheres", "scene_tabletop", "scene_uniform", "batch_maps",
    "look_at", "poses_sphere", "poses_shell", "poses_ball", "trajectories_walk",
    "Camera", "Workload", "make_config", "scene_seed", "pose_seed",
]
