"""ctypes front-end of the C oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

RAY_MISS, RAY_HIT, RAY_END, RAY_EXIT, RAY_INVALID = 0, 1, 2, 3, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbt_oracle.c")
_LIB = os.path.join(_HERE, "libnbt_oracle.so")
_CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared"]
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary32 geometry, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleMap(C.Structure):
    _fields_ = [("P", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("voxel", C.c_float), ("origin", C.c_float * 3),
                ("occ_threshold", C.c_float), ("free_threshold", C.c_float)]


class OracleCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tan_half_h", C.c_float),
                ("tan_half_v", C.c_float), ("range", C.c_float)]


class OracleRay(C.Structure):
    _fields_ = [("steps", C.c_uint32), ("stop_lin", C.c_int32), ("reason", C.c_int32),
                ("hash", C.c_uint64), ("gain", C.c_double)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = C.CDLL(_LIB)
            L.oracle_fnv1a_bytes.restype = C.c_uint64
            L.oracle_fnv1a_bytes.argtypes = [C.c_void_p, C.c_int64]
            L.oracle_cast_ray.restype = None
            L.oracle_cast_ray.argtypes = [C.POINTER(OracleMap), C.POINTER(OracleCamera), C.c_void_p,
                                          C.c_int, C.c_int, C.c_void_p, C.c_int, C.POINTER(OracleRay)]
            L.oracle_trace_rays.restype = None
            L.oracle_trace_rays.argtypes = [C.POINTER(OracleMap), C.POINTER(OracleCamera), C.c_void_p,
                                            C.c_int64] + [C.c_void_p] * 5
            L.oracle_eval_viewpoints.restype = None
            L.oracle_eval_viewpoints.argtypes = [C.POINTER(OracleMap), C.POINTER(OracleCamera),
                                                 C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
            L.oracle_eval_trajectories.restype = C.c_int
            L.oracle_eval_trajectories.argtypes = [C.POINTER(OracleMap), C.POINTER(OracleCamera),
                                                   C.c_void_p, C.c_int64, C.c_int64,
                                                   C.c_void_p, C.c_void_p, C.c_void_p]
            L.oracle_insert_scans.restype = C.c_int
            L.oracle_insert_scans.argtypes = [C.POINTER(OracleMap), C.POINTER(OracleCamera),
                                              C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                                              C.c_float, C.c_float, C.c_float, C.c_void_p]
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class _MapRef:
    """Keeps the probability array alive while the C struct points at it."""

    def __init__(self, P, voxel, origin, occ_threshold=0.5, free_threshold=0.5):
        self.P = np.ascontiguousarray(P, dtype=np.float32)
        nz, ny, nx = self.P.shape
        o = np.asarray(origin, dtype=np.float32)
        self.s = OracleMap(_ptr(self.P).value, nx, ny, nz, float(np.float32(voxel)),
                           (C.c_float * 3)(*[float(v) for v in o]),
                           float(np.float32(occ_threshold)), float(np.float32(free_threshold)))


def _map(scene_or_P, voxel=None, origin=None, occ_threshold=0.5, free_threshold=0.5):
    if hasattr(scene_or_P, "P"):
        s = scene_or_P
        return _MapRef(s.P, s.voxel, s.origin, occ_threshold, free_threshold)
    return _MapRef(scene_or_P, voxel, origin, occ_threshold, free_threshold)


def _cam(camera):
    if hasattr(camera, "as_tuple"):
        w, h, th, tv, r = camera.as_tuple()
    else:
        w, h, th, tv, r = camera
    return OracleCamera(int(w), int(h), float(np.float32(th)), float(np.float32(tv)),
                        float(np.float32(r)))


def fnv1a(data: bytes) -> int:
    buf = np.frombuffer(bytes(data), dtype=np.uint8).copy()
    return int(lib().oracle_fnv1a_bytes(_ptr(buf), len(buf)))


def cast_ray(scene, camera, pose, i, j, thresholds=(0.5, 0.5), with_path=True):
    """One ray: returns dict(steps, stop_lin, reason, hash, gain, path)."""
    m = _map(scene, occ_threshold=thresholds[0], free_threshold=thresholds[1])
    cam = _cam(camera)
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    nx, ny, nz = m.s.nx, m.s.ny, m.s.nz
    cap = nx + ny + nz + 3
    path = np.full(cap, -1, dtype=np.int32)
    r = OracleRay()
    lib().oracle_cast_ray(C.byref(m.s), C.byref(cam), _ptr(pose), int(i), int(j),
                          _ptr(path) if with_path else None, cap, C.byref(r))
    return {"steps": int(r.steps), "stop_lin": int(r.stop_lin), "reason": int(r.reason),
            "hash": int(r.hash), "gain": float(r.gain),
            "path": path[: min(int(r.steps), cap)].copy() if with_path else None}


def trace_rays(scene, camera, poses, thresholds=(0.5, 0.5)):
    """Per-ray digests for every pose: dict of arrays shaped [N, H*W]."""
    m = _map(scene, occ_threshold=thresholds[0], free_threshold=thresholds[1])
    cam = _cam(camera)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    n = poses.shape[0]
    rays = cam.width * cam.height
    out = {"steps": np.zeros((n, rays), np.uint32), "stop_lin": np.zeros((n, rays), np.int32),
           "reason": np.zeros((n, rays), np.int32), "hash": np.zeros((n, rays), np.uint64),
           "gain": np.zeros((n, rays), np.float64)}
    lib().oracle_trace_rays(C.byref(m.s), C.byref(cam), _ptr(poses), n, _ptr(out["steps"]),
                            _ptr(out["stop_lin"]), _ptr(out["reason"]), _ptr(out["hash"]),
                            _ptr(out["gain"]))
    return out


def eval_viewpoints(scene, camera, poses, thresholds=(0.5, 0.5)):
    """Per-perspective IG (float32) and total voxel steps (uint64)."""
    m = _map(scene, occ_threshold=thresholds[0], free_threshold=thresholds[1])
    cam = _cam(camera)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    n = poses.shape[0]
    ig = np.zeros(n, np.float32)
    steps = np.zeros(n, np.uint64)
    lib().oracle_eval_viewpoints(C.byref(m.s), C.byref(cam), _ptr(poses), n, _ptr(ig), _ptr(steps))
    return ig, steps


def eval_trajectories(scene, camera, poses, thresholds=(0.5, 0.5)):
    """Per-trajectory union IG, counts [T,4] (unique, occ, free, unknown) and visits."""
    m = _map(scene, occ_threshold=thresholds[0], free_threshold=thresholds[1])
    cam = _cam(camera)
    poses = np.ascontiguousarray(poses, dtype=np.float32)
    T, L = poses.shape[0], poses.shape[1]
    ig = np.zeros(T, np.float32)
    counts = np.zeros((T, 4), np.uint32)
    visits = np.zeros(T, np.uint64)
    rc = lib().oracle_eval_trajectories(C.byref(m.s), C.byref(cam), _ptr(poses), T, L,
                                        _ptr(ig), _ptr(counts), _ptr(visits))
    if rc != 0:
        raise MemoryError("oracle_eval_trajectories: out of memory")
    return ig, counts, visits


# Log-odds increments and clamping bounds of the occupancy update: the common
# defaults of octree occupancy maps (hit 0.7, miss 0.4, clamped to
# [0.1192, 0.971] in probability), as binary32 log-odds.
DEFAULT_INSERT_PARAMS = tuple(float(np.float32(np.log(p / (1.0 - p)))) for p in (0.7, 0.4, 0.1192, 0.971))


def insert_scans(geometry, camera, poses, depth, logodds, params=DEFAULT_INSERT_PARAMS):
    """Depth-image insertion (I1-I5 of nbt_oracle.c): returns the updated copy of ``logodds``
    [nz, ny, nx].  ``geometry`` supplies the grid (its P only for the shape), ``poses`` [K, 12],
    ``depth`` [K, H, W] z-depths in metres; ``params`` = (l_hit, l_miss, l_min, l_max)."""
    L = np.array(logodds, dtype=np.float32, copy=True, order="C")
    m = _map(geometry) if hasattr(geometry, "P") else _map(L, *geometry)
    cam = _cam(camera)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    depth = np.ascontiguousarray(depth, dtype=np.float32).reshape(poses.shape[0], cam.height, cam.width)
    assert L.shape == (m.s.nz, m.s.ny, m.s.nx)
    hit, miss, lo, hi = (float(np.float32(v)) for v in params)
    rc = lib().oracle_insert_scans(C.byref(m.s), C.byref(cam), _ptr(poses), _ptr(depth), poses.shape[0],
                                   hit, miss, lo, hi, _ptr(L))
    if rc != 0:
        raise MemoryError("oracle_insert_scans: out of memory")
    return L


def logodds_to_prob(L):
    """P = 1 / (1 + exp(-L)) in binary64, rounded once to binary32."""
    L = np.asarray(L, dtype=np.float64)
    return (1.0 / (1.0 + np.exp(-L))).astype(np.float32)
