"""Pins of the oracle's depth-image insertion (log-odds occupancy update, I1-I5 of nbt_oracle.c).

Each pin is fixed by geometry or by the update rule itself, not by re-running the oracle's code:
hand-placed rays along one map row, the clamping bounds reached after repeated scans, the
return point's voxel computed in binary64 from the pose, and agreement of the carved voxels
with the (separately pinned) ray walk of oracle.cast_ray.
"""

import numpy as np
import pytest

import oracle
from workloads import look_at, poses_sphere, scene_spheres
from workloads.configs import Camera

HIT, MISS, LMIN, LMAX = (np.float32(v) for v in oracle.DEFAULT_INSERT_PARAMS)


def _row_setup(width=1, fov=0.001):
    """8x1x1 map of 1 m voxels; camera 1.5 m before its x = 0 face looking along +x through the
    voxel centres (y = z = 0.5); z-depth d puts the return at x = d - 1.5."""
    geom = (1.0, np.zeros(3, np.float32))
    L = np.zeros((1, 1, 8), np.float32)
    cam = Camera(width, 1, fov, fov, 20.0)
    pose = look_at(np.array([[-1.5, 0.5, 0.5]]), np.array([10.0, 0.5, 0.5]))
    return geom, L, cam, pose


def _insert(geom, L, cam, poses, depth, params=oracle.DEFAULT_INSERT_PARAMS):
    return oracle.insert_scans(geom, cam, poses, np.asarray(depth, np.float32), L, params)


def test_params_are_the_log_odds_of_the_usual_probabilities():
    for l, p in zip((HIT, MISS, LMIN, LMAX), (0.7, 0.4, 0.1192, 0.971)):
        assert abs(1.0 / (1.0 + np.exp(-float(l))) - p) < 1e-6


def test_single_ray_free_then_hit():
    geom, L, cam, pose = _row_setup()
    out = _insert(geom, L, cam, pose, [[[5.2]]])                 # return at x = 3.7: voxel 3
    assert out[0, 0].tolist() == [MISS, MISS, MISS, HIT, 0, 0, 0, 0]


@pytest.mark.parametrize("d", [np.inf, 20.0, 30.0])
def test_no_return_within_range_carves_free(d):
    geom, L, cam, pose = _row_setup()
    out = _insert(geom, L, cam, pose, [[[d]]])
    assert out[0, 0].tolist() == [MISS] * 8


def test_depth_exactly_at_range_is_no_return():
    # a 24-voxel row holds the far-plane endpoint (x = 18.5): depth = range carves the row up
    # to the endpoint's voxel but marks no hit there
    geom = (1.0, np.zeros(3, np.float32))
    L = np.zeros((1, 1, 24), np.float32)
    cam = Camera(1, 1, 0.001, 0.001, 20.0)
    pose = look_at(np.array([[-1.5, 0.5, 0.5]]), np.array([30.0, 0.5, 0.5]))
    out = _insert(geom, L, cam, pose, [[[20.0]]])
    assert out[0, 0].tolist() == [MISS] * 19 + [0] * 5
    out = _insert(geom, L, cam, pose, [[[19.9]]])              # just inside range: a return
    assert out[0, 0].tolist() == [MISS] * 18 + [HIT] + [0] * 5


@pytest.mark.parametrize("d", [0.0, -1.0, np.nan])
def test_no_measurement_changes_nothing(d):
    geom, L, cam, pose = _row_setup()
    out = _insert(geom, L, cam, pose, [[[d]]])
    assert not out.any()


def test_return_beyond_or_before_the_map():
    geom, L, cam, pose = _row_setup()
    beyond = _insert(geom, L, cam, pose, [[[12.0]]])             # x = 10.5, past the last voxel
    assert beyond[0, 0].tolist() == [MISS] * 8
    before = _insert(geom, L, cam, pose, [[[1.0]]])              # x = -0.5, before the map
    assert not before.any()


def test_repeated_scans_reach_the_clamping_bounds():
    geom, L, cam, pose = _row_setup()
    poses = np.repeat(pose, 10, axis=0)
    out = _insert(geom, L, cam, poses, np.full((10, 1, 1), 5.2, np.float32))
    assert out[0, 0].tolist() == [LMIN, LMIN, LMIN, LMAX, 0, 0, 0, 0]


def test_hit_wins_and_each_voxel_changes_once_per_scan():
    # two nearly coincident rays: one returns in voxel 3, the other in voxel 6 and passes
    # voxel 3; three more copies of the scan's rays would not change a discrete update
    geom, L, cam, pose = _row_setup(width=2)
    out = _insert(geom, L, cam, pose, [[[5.2, 7.9]]])
    assert out[0, 0].tolist() == [MISS, MISS, MISS, HIT, MISS, MISS, HIT, 0]
    geom, L, cam4, pose = _row_setup(width=4)
    out4 = _insert(geom, L, cam4, pose, [[[5.2, 7.9, 5.2, 7.9]]])
    assert np.array_equal(out4, out)


def test_scan_order_does_not_matter_without_clamping():
    sc = scene_spheres(n=(24, 20, 16), voxel=0.1, n_spheres=0, seed=71)
    cam = Camera(9, 7, 50.0, 40.0, 3.0)
    poses = poses_sphere(sc.poi, 0.8, 2, seed=72)
    rng = np.random.default_rng(73)
    depth = rng.uniform(0.3, 2.5, size=(2, 7, 9)).astype(np.float32)
    L0 = np.zeros(sc.P.shape, np.float32)
    ab = oracle.insert_scans(sc, cam, poses, depth, L0)
    ba = oracle.insert_scans(sc, cam, poses[::-1].copy(), depth[::-1].copy(), L0)
    assert np.array_equal(ab, ba) and ab.any()


def test_carved_voxels_are_the_cast_ray_paths_and_hits_hold_the_return_point():
    sc = scene_spheres(n=(32, 28, 24), voxel=0.05, n_spheres=0, seed=81)
    sc.P[:] = np.float32(0.2)                  # all free: cast_ray walks each segment to its end
    cam = Camera(11, 9, 60.0, 45.0, 1.5)
    poses = poses_sphere(sc.poi, 0.5, 3, seed=82)
    L0 = np.zeros(sc.P.shape, np.float32)
    # no returns: the carved set is the union of the walks of cast_ray
    out = oracle.insert_scans(sc, cam, poses[:1], np.full((1, 9, 11), np.inf, np.float32), L0)
    walked = set()
    for j in range(9):
        for i in range(11):
            walked.update(int(v) for v in oracle.cast_ray(sc, cam, poses[0], i, j)["path"])
    assert set(np.flatnonzero(out.ravel()).tolist()) == walked
    assert np.all(out.ravel()[list(walked)] == MISS)
    # returns inside the map: the hit voxel holds the return point (computed in binary64)
    rng = np.random.default_rng(83)
    depth = rng.uniform(0.2, 0.9, size=(1, 9, 11)).astype(np.float32) * np.float32(cam.range)
    out = oracle.insert_scans(sc, cam, poses[1:2], depth, L0)
    pose = poses[1].astype(np.float64)
    R, t = pose[:9].reshape(3, 3), pose[9:]
    nz, ny, nx = sc.P.shape
    checked = 0
    for j in range(9):
        for i in range(11):
            u = cam.range * float(cam.tan_h) * (2 * i - 10) / 10
            v = cam.range * float(cam.tan_v) * (2 * j - 8) / 8
            s = float(depth[0, j, i]) / cam.range
            p = t + R @ (s * np.array([u, v, cam.range]))
            q = (p - sc.origin.astype(np.float64)) / sc.voxel
            f = np.floor(q)
            if np.any(np.abs(q - np.round(q)) < 1e-3) or np.any(f < 0) or np.any(f >= (nx, ny, nz)):
                continue                       # too close to a face, or outside the map
            lin = (int(f[2]) * ny + int(f[1])) * nx + int(f[0])
            assert out.ravel()[lin] == HIT, (i, j)
            checked += 1
    assert checked >= 50


def test_logodds_to_prob_closed_forms():
    """The logistic at points where it has an exact rational value: L = 0 -> 1/2,
    L = +-ln 3 -> 3/4 and 1/4, L = ln(7/3) -> 7/10, L = ln 9 -> 9/10 (each the binary32
    nearest the rational), the limits for large |L|, and P(L) + P(-L) = 1."""
    import math
    pts = {0.0: 0.5, math.log(3.0): 0.75, -math.log(3.0): 0.25, math.log(7.0 / 3.0): 0.7,
           math.log(9.0): 0.9, -math.log(9.0): 0.1}
    got = oracle.logodds_to_prob(np.array(list(pts.keys())))
    assert got.dtype == np.float32
    assert got.tolist() == [float(np.float32(v)) for v in pts.values()]
    big = oracle.logodds_to_prob(np.array([100.0, 1e4, -1e4, -100.0]))
    assert big[0] == 1.0 and big[1] == 1.0 and big[2] == 0.0
    assert 0.0 < big[3] < 1e-43                         # e^-100 ~ 3.7e-44: a binary32 subnormal
    L = np.linspace(-12.0, 12.0, 97)
    s = oracle.logodds_to_prob(L).astype(np.float64) + oracle.logodds_to_prob(-L).astype(np.float64)
    assert np.all(np.abs(s - 1.0) <= 2.0 ** -24)
    assert np.all(np.diff(oracle.logodds_to_prob(L).astype(np.float64)) > 0)
