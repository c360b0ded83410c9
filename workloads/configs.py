"""The benchmark workloads: scenes, cameras and poses for the five configurations.

==== =========================================================================
cfg  workload
==== =========================================================================
1    64^3 map, 5 cm voxels, 20 spheres; 32 viewpoints on a 0.8 m sphere;
     64x48 rays, 60x45 deg, 2 m range
2    256^3 map, 2 cm voxels, table-top clutter (200 objects, 3 prior views);
     4 PoIs x 1024 viewpoints in the 0.5-1.2 m shell; 160x120 rays,
     70x55 deg, 3 m range
3    64 sphere maps with edge in {64,96,128,192,256}, 5 cm voxels; per-map
     viewpoint count log-uniform in [16, 2048] on the 0.8 m sphere; camera of cfg 1
4    256^3 sphere map (5 cm voxels, sphere count scaled by volume);
     4096 trajectories x 24 poses on the 0.6-1.0 m shell; 128x96 rays,
     60x45 deg, 2 m range
==== =========================================================================

``scale`` shrinks viewpoint / trajectory counts for tests (maps are kept).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .poses import poses_shell, poses_sphere, trajectories_walk
from .scenes import SceneMap, batch_maps, scene_spheres, scene_tabletop


def scene_seed(cfg: int, map_idx: int = 0) -> int:
    return 22588 + 1000 * cfg + map_idx


def pose_seed(cfg: int, map_idx: int = 0) -> int:
    return scene_seed(cfg, map_idx) + 500


@dataclass
class Camera:
    """Pinhole camera as the far-plane ray grid of Sec. III (endpoint calculation).

    ``width x height`` endpoints on the far plane at depth ``range``; the
    half-extents are ``range * tan(fov/2)``.  The tangents are evaluated in
    double precision and rounded once to float32 so that every consumer sees
    the same bits.
    """

    width: int
    height: int
    fov_h_deg: float
    fov_v_deg: float
    range: float

    @property
    def tan_h(self) -> np.float32:
        return np.float32(math.tan(math.radians(self.fov_h_deg) / 2.0))

    @property
    def tan_v(self) -> np.float32:
        return np.float32(math.tan(math.radians(self.fov_v_deg) / 2.0))

    @property
    def rays(self) -> int:
        return self.width * self.height

    def as_tuple(self):
        return (int(self.width), int(self.height), float(self.tan_h), float(self.tan_v),
                float(np.float32(self.range)))


CAM1 = Camera(64, 48, 60.0, 45.0, 2.0)
CAM2 = Camera(160, 120, 70.0, 55.0, 3.0)
CAM4 = Camera(128, 96, 60.0, 45.0, 2.0)


@dataclass
class Workload:
    cfg: int
    name: str
    maps: list                     # list[SceneMap]
    camera: Camera
    poses: list                    # per map: float32 [N, 12]   (cfg 4: [T, L, 12])
    meta: dict = field(default_factory=dict)

    @property
    def n_viewpoints(self) -> int:
        return int(sum(p.shape[0] for p in self.poses))


def make_config(cfg: int, scale: float = 1.0, n_maps: int | None = None) -> Workload:
    if cfg == 1:
        m = scene_spheres(n=64, voxel=0.05, n_spheres=20, seed=scene_seed(1))
        n = max(1, int(round(32 * scale)))
        poses = poses_sphere(m.poi, 0.8, n, pose_seed(1))
        return Workload(1, "plain raycast 64^3 spheres", [m], CAM1, [poses])
    if cfg == 2:
        m = scene_tabletop(n=256, voxel=0.02, n_objects=200, seed=scene_seed(2))
        tops = m.extra["object_tops"]
        rng = np.random.Generator(np.random.PCG64(pose_seed(2)))
        pick = rng.choice(len(tops), size=4, replace=False)
        per = max(1, int(round(1024 * scale)))
        chunks = [poses_shell(tops[k], 0.5, 1.2, per, pose_seed(2, 1 + i)) for i, k in enumerate(pick)]
        poses = np.concatenate(chunks, axis=0)
        return Workload(2, "plain raycast 256^3 table-top", [m], CAM2, [poses],
                        meta={"pois": tops[pick], "per_poi": per})
    if cfg == 3:
        maps = batch_maps(n_maps=64 if n_maps is None else n_maps, voxel=0.05, cfg=3)
        rng = np.random.Generator(np.random.PCG64(pose_seed(3, 999)))
        counts = np.floor(np.exp(rng.uniform(math.log(16), math.log(2048), size=len(maps))))
        counts = np.maximum(1, np.round(counts * scale)).astype(int)
        poses = [poses_sphere(m.poi, 0.8, int(c), pose_seed(3, i)) for i, (m, c) in enumerate(zip(maps, counts))]
        return Workload(3, "batched 64 maps", maps, CAM1, poses)
    if cfg == 4:
        m = scene_spheres(n=256, voxel=0.05, n_spheres=1280, seed=scene_seed(4))
        t = max(1, int(round(4096 * scale)))
        traj = trajectories_walk(m.poi, t, 24, pose_seed(4))
        return Workload(4, "trajectory IG 256^3", [m], CAM4, [traj])
    raise ValueError(f"unknown config {cfg}")
