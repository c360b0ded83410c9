"""The seeded input generators (no GPU): determinism per seed, the geometry of the sampled
poses (orthonormal look-at frames, Eq. 1's ball, the shells and spheres of the benchmark
configurations, the smooth trajectory walks) and the occupancy statistics of the scenes."""

import math

import numpy as np
import pytest
from scipy import stats

from workloads import (batch_maps, look_at, make_config, poses_ball, poses_shell, poses_sphere,
                       scene_spheres, scene_tabletop, trajectories_walk)
from workloads.scenes import P_FREE, P_OCC, P_UNKNOWN


def _frames(poses):
    R = poses[..., :9].astype(np.float64).reshape(-1, 3, 3)
    t = poses[..., 9:].astype(np.float64).reshape(-1, 3)
    return R, t


def _assert_look_at(poses, poi, tol=2e-6):
    R, t = _frames(poses)
    eye = np.einsum("nij,nik->njk", R, R)
    assert np.abs(eye - np.eye(3)).max() < tol                    # orthonormal columns
    assert np.abs(np.linalg.det(R) - 1.0).max() < tol             # right-handed, no reflection
    view = np.asarray(poi, np.float64) - t
    d = np.linalg.norm(view, axis=1)
    ok = d > 1e-9
    cosang = np.einsum("ni,ni->n", R[ok][:, :, 2], view[ok] / d[ok, None])
    assert cosang.min() > 1.0 - 1e-6                              # camera z looks at the PoI
    # roll: camera x horizontal unless the view is near vertical
    vert = np.abs(R[:, 2, 2]) > 0.9999
    assert np.abs(R[~vert][:, 2, 0]).max() < tol


@pytest.mark.parametrize("gen", ["sphere", "shell", "ball"])
def test_pose_samplers_deterministic_per_seed(gen):
    poi = np.array([0.3, -0.2, 1.1])
    f = {"sphere": lambda s: poses_sphere(poi, 0.8, 257, s), "shell": lambda s: poses_shell(poi, 0.5, 1.2, 257, s),
         "ball": lambda s: poses_ball(poi, 1.0, 257, s)}[gen]
    a, b, c = f(11), f(11), f(12)
    assert a.dtype == np.float32 and a.shape == (257, 12)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_look_at_frames():
    rng = np.random.default_rng(3)
    pos = rng.normal(size=(500, 3))
    pos[0] = (0.0, 0.0, 5.0)                      # straight above: the +Y fallback
    pos[1] = (0.0, 0.0, -5.0)                     # straight below
    poi = np.zeros(3)
    p = look_at(pos, poi)
    _assert_look_at(p, poi)
    R, _ = _frames(p[:2])
    assert np.allclose(R[0][:, 2], (0, 0, -1), atol=1e-7) and np.allclose(R[1][:, 2], (0, 0, 1), atol=1e-7)
    # a camera at its target looks straight down
    R0, _ = _frames(look_at(np.zeros((1, 3)), np.zeros(3)))
    assert np.allclose(R0[0][:, 2], (0, 0, -1))


def test_poses_ball_is_uniform_in_the_ball():
    """Eq. 1 (read with a U(0,1) radial draw and the PoI offset): every start point lies in the
    ball of radius r_S, (r / r_S)^3 is U(0,1) (Kolmogorov-Smirnov), directions are isotropic
    (mean unit vector near 0, each coordinate of a unit vector U(-1,1)), and every pose looks
    at the PoI."""
    poi = np.array([1.2, 0.7, 0.9])
    r_s, n = 1.0, 20000
    p = poses_ball(poi, r_s, n, seed=4242)
    _, t = _frames(p)
    v = t - poi
    r = np.linalg.norm(v, axis=1)
    assert r.max() <= r_s * (1 + 1e-6)
    assert stats.kstest((r / r_s) ** 3, "uniform").pvalue > 1e-3
    u = v / r[:, None]
    assert np.linalg.norm(u.mean(axis=0)) < 4.0 / math.sqrt(n)
    for a in range(3):
        assert stats.kstest((u[:, a] + 1) / 2, "uniform").pvalue > 1e-3
    # a radius-only sampler on the sphere would fail the volume law
    assert stats.kstest(np.ones(n), "uniform").pvalue < 1e-6
    _assert_look_at(p, poi)


def test_poses_shell_and_sphere_radii():
    poi = np.array([0.0, 0.0, 0.0])
    p = poses_shell(poi, 0.5, 1.2, 20000, seed=7)
    r = np.linalg.norm(_frames(p)[1] - poi, axis=1)
    assert r.min() >= 0.5 - 1e-6 and r.max() <= 1.2 + 1e-6
    assert stats.kstest((r ** 3 - 0.5 ** 3) / (1.2 ** 3 - 0.5 ** 3), "uniform").pvalue > 1e-3
    _assert_look_at(p, poi)
    s = poses_sphere(poi, 0.8, 5000, seed=8)
    rs = np.linalg.norm(_frames(s)[1] - poi, axis=1)
    assert np.abs(rs - 0.8).max() < 1e-6
    _assert_look_at(s, poi)


def test_trajectory_walk_geometry():
    """3 cm steps (plus the radial jitter), radius kept in [0.6, 1.0] m, and the viewing axis
    within the 15 degree offset bound of the look-at direction."""
    poi = np.array([6.4, 6.4, 6.4])
    tr = trajectories_walk(poi, 200, 24, seed=99)
    assert tr.shape == (200, 24, 12) and tr.dtype == np.float32
    assert np.array_equal(tr, trajectories_walk(poi, 200, 24, seed=99))
    R, t = _frames(tr)
    t = t.reshape(200, 24, 3)
    r = np.linalg.norm(t - poi, axis=2)
    assert r.min() >= 0.6 - 1e-5 and r.max() <= 1.0 + 1e-5
    step = np.linalg.norm(np.diff(t, axis=1), axis=2)
    assert step.min() > 0.02 and step.max() < 0.045
    view = (poi - t.reshape(-1, 3))
    view /= np.linalg.norm(view, axis=1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip(np.einsum("ni,ni->n", R[:, :, 2], view), -1, 1)))
    assert ang.max() <= 15.0 + 1e-3
    eye = np.einsum("nij,nik->njk", R, R)
    assert np.abs(eye - np.eye(3)).max() < 2e-6


def test_sphere_scene_matches_its_definition():
    """Small map: the occupied voxels are exactly those whose centre lies in one of the drawn
    balls (brute force over every voxel centre), the rest split free / unknown by the plane
    through the PoI; deterministic per seed."""
    sc = scene_spheres(n=(20, 18, 16), voxel=0.05, n_spheres=6, seed=31, origin=(0.1, -0.2, 0.3))
    again = scene_spheres(n=(20, 18, 16), voxel=0.05, n_spheres=6, seed=31, origin=(0.1, -0.2, 0.3))
    assert np.array_equal(sc.P, again.P)
    nz, ny, nx = sc.P.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cen = np.stack([x, y, z], axis=-1) * sc.voxel + sc.voxel / 2 + sc.origin.astype(np.float64)
    occ = np.zeros(sc.P.shape, bool)
    for c, r in zip(sc.extra["sphere_centres"], sc.extra["sphere_radii"]):
        occ |= np.sum((cen - c) ** 2, axis=-1) <= r * r
    assert np.array_equal(sc.P == P_OCC, occ)
    side = (cen - sc.poi) @ sc.extra["normal"]
    assert np.array_equal(sc.P[~occ] == P_FREE, side[~occ] > 0)
    assert np.array_equal(sc.P[~occ] == P_UNKNOWN, ~(side[~occ] > 0))


def test_config1_occupancy_and_counts():
    """Config 1: 20 balls of 5-15 cm in a 64^3 map at 5 cm occupy a few tenths of a percent
    (the count and radii fix it; a '3 %' reading would need ten times the volume), the free /
    unknown split of the remainder is near half and half, 32 perspectives on the 0.8 m sphere."""
    w = make_config(1)
    f = w.maps[0].fractions()
    assert 0.001 < f["occupied"] < 0.01
    assert 0.25 < f["free"] < 0.75 and abs(sum(f.values()) - 1.0) < 1e-12
    assert w.poses[0].shape == (32, 12)
    r = np.linalg.norm(_frames(w.poses[0])[1] - w.maps[0].poi, axis=1)
    assert np.abs(r - 0.8).max() < 1e-6


def test_tabletop_scene_states():
    """A small table-top: three states only, the unknown region non-empty (space hidden from
    the prior cameras), occupied voxels only at or above the table slab, object tops above
    the table, deterministic per seed."""
    sc = scene_tabletop(n=96, voxel=0.02, n_objects=20, seed=77)
    vals = set(np.unique(sc.P).tolist())
    assert vals <= {float(P_OCC), float(P_FREE), float(P_UNKNOWN)}
    f = sc.fractions()
    assert f["unknown"] > 0.001 and f["free"] > 0.5 and f["occupied"] > 0.0001
    occ_z = np.nonzero(sc.P == P_OCC)[0]
    table_iz = int(np.floor(sc.extra["table_z"] / sc.voxel))
    assert occ_z.min() >= table_iz - 3
    assert np.all(sc.extra["object_tops"][:, 2] > sc.extra["table_z"])
    assert np.array_equal(sc.P, scene_tabletop(n=96, voxel=0.02, n_objects=20, seed=77).P)


def test_batch_maps_sizes_and_seeds():
    maps = batch_maps(n_maps=6, sizes=(16, 24), voxel=0.05, cfg=9, base_spheres=20)
    assert all(m.P.shape[0] in (16, 24) and m.P.shape[0] == m.P.shape[1] == m.P.shape[2] for m in maps)
    again = batch_maps(n_maps=6, sizes=(16, 24), voxel=0.05, cfg=9, base_spheres=20)
    assert all(np.array_equal(a.P, b.P) for a, b in zip(maps, again))
    assert not np.array_equal(maps[0].P, maps[1].P) or maps[0].P.shape != maps[1].P.shape


def test_surrogate_training_maps_roundtrip():
    """The table-top surrogate's trainer ships maps as one code per voxel: the codes give back
    the generator's probabilities exactly, and the PoIs are object tops of that map."""
    from paper_2503_22588_amd import train_surrogate as T
    codes, tops = T.tabletop_scene(22588 + 6000, n_pois=4)
    sc = scene_tabletop(n=256, voxel=0.02, n_objects=200, seed=22588 + 6000)
    assert codes.dtype == np.uint8 and np.array_equal(T.P_CODES[codes], sc.P)
    assert tops.shape == (4, 3)
    assert all(np.any(np.all(np.isclose(sc.extra["object_tops"], t, atol=1e-6), axis=1)) for t in tops)
