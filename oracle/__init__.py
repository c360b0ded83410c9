"""CPU oracle for information-gain raycasting -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The GPU library never links, calls
or reads anything here, and nothing here imports the library.

``nbt_oracle.c`` is the plain single-threaded definition of the method
(Sec. III of the paper: endpoint grid, Eq. 2 voxel gains, the first-occupied
stop rule and the per-perspective mean), plus the per-trajectory union and the
log-odds map update from depth images that precedes IG evaluation.
``surrogate.py`` holds the float64 NumPy forward pass of the learned IG
surrogate and ``idw.py`` the planner-side interpolation of Eq. 3.
"""

from .oracle import (
    RAY_MISS, RAY_HIT, RAY_END, RAY_EXIT, RAY_INVALID,
    OracleMap, OracleCamera, build, lib,
    cast_ray, trace_rays, eval_viewpoints, eval_trajectories, fnv1a,
    insert_scans, logodds_to_prob, DEFAULT_INSERT_PARAMS,
)

__all__ = [
    "RAY_MISS", "RAY_HIT", "RAY_END", "RAY_EXIT", "RAY_INVALID",
    "OracleMap", "OracleCamera", "build", "lib",
    "cast_ray", "trace_rays", "eval_viewpoints", "eval_trajectories", "fnv1a",
    "insert_scans", "logodds_to_prob", "DEFAULT_INSERT_PARAMS",
]
