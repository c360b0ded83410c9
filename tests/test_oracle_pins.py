"""Pins of the CPU oracle against what the paper and geometry fix (no GPU).

Each test checks the oracle against something other than itself: the cases
of Eq. 2, hand-worked rays, exact rational segment/voxel intersection on tiny
maps, closed forms for uniform maps, slabs and spheres, and structural
invariants of a voxel walk.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import look_at, scene_uniform, scene_spheres, poses_sphere
from workloads.configs import Camera

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32 = np.float32
REASON = {"MISS": 0, "HIT": 1, "END": 2, "EXIT": 3, "INVALID": 4}


def _scene(P, voxel=1.0, origin=(0, 0, 0)):
    class S:
        pass
    s = S()
    s.P = np.ascontiguousarray(P, dtype=np.float32)
    s.voxel = voxel
    s.origin = np.asarray(origin, dtype=np.float32)
    return s


def _axis_pose(t, direction):
    """Pose whose optical axis (third rotation column) is ``direction`` exactly."""
    d = np.asarray(direction, dtype=np.float32)
    p = look_at(np.asarray(t, np.float64)[None], np.asarray(t, np.float64) + d.astype(np.float64))[0]
    p[2], p[5], p[8] = d[0], d[1], d[2]
    p[9:] = np.asarray(t, dtype=np.float32)
    return p


def _lin_to_xyz(lin, nx, ny):
    return lin % nx, (lin // nx) % ny, lin // (nx * ny)


# ---------------------------------------------------------------- Eq. 2 -----

@pytest.mark.parametrize("p,thr,expected_gain,is_hit", [
    (0.9, (0.5, 0.5), float(F32(1) - F32(0.9)), True),      # occupied: 1 - P
    (1.0, (0.5, 0.5), 0.0, True),                           # certain occupied: nothing left to gain
    (0.2, (0.5, 0.5), float(F32(0.2)), False),              # free: P
    (0.0, (0.5, 0.5), 0.0, False),                          # certain free
    (0.5, (0.5, 0.5), 1.0, False),                          # unknown: 1
    (0.6, (0.7, 0.3), 1.0, False),                          # between thresholds: unknown
    (0.75, (0.7, 0.3), float(F32(1) - F32(0.75)), True),
    (0.25, (0.7, 0.3), float(F32(0.25)), False),
])
def test_eq2_single_voxel(oracle_lib, p, thr, expected_gain, is_hit):
    """Camera inside a 1-voxel map: the ray sees exactly that voxel (Eq. 2 cases)."""
    s = _scene(np.full((1, 1, 1), p))
    pose = _axis_pose((0.5, 0.5, 0.5), (1.0, 0.0, 0.0))
    r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 5.0), pose, 0, 0, thresholds=thr)
    assert r["steps"] == 1
    assert r["gain"] == expected_gain
    assert r["reason"] == (oracle.RAY_HIT if is_hit else oracle.RAY_EXIT)


# ------------------------------------------------------- hand-worked rays ---

def test_hand_worked_fixtures(oracle_lib):
    data = json.load(open(os.path.join(GOLDEN, "hand_worked.json")))
    for case in data["cases"]:
        nx, ny, nz = case["dims"]
        P = np.asarray(case["P"], dtype=np.float32).reshape(nz, ny, nx)
        s = _scene(P)
        c = case["camera"]
        cam = (c["width"], c["height"], c["tan_half_h"], c["tan_half_v"], c["range"])
        pose = np.asarray(case["pose"], dtype=np.float32)
        for ray in case["rays"]:
            r = oracle.cast_ray(s, cam, pose, ray["i"], ray["j"])
            assert list(r["path"]) == ray["path"], case["name"]
            assert r["reason"] == REASON[ray["reason"]], case["name"]
            assert r["gain"] == pytest.approx(ray["gain"], rel=0, abs=1e-15), case["name"]
        ig, steps = oracle.eval_viewpoints(s, cam, pose[None])
        assert float(ig[0]) == float(np.float32(case["ig"])), case["name"]
        assert int(steps[0]) == sum(len(r["path"]) for r in case["rays"])


def test_fnv1a_published_vectors(oracle_lib):
    # FNV-1a 64-bit test vectors: "" -> offset basis, "a" -> 0xaf63dc4c8601ec8c
    assert oracle.fnv1a(b"") == 0xcbf29ce484222325
    assert oracle.fnv1a(b"a") == 0xaf63dc4c8601ec8c
    assert oracle.fnv1a(b"foobar") == 0x85944171f73967e8


def test_digest_hash_is_fnv_of_path(oracle_lib):
    w = scene_spheres(n=24, voxel=0.1, n_spheres=6, seed=7)
    poses = poses_sphere(w.poi, 0.6, 3, seed=8)
    cam = Camera(9, 7, 60, 45, 1.5)
    for p in poses:
        for (i, j) in [(0, 0), (4, 3), (8, 6)]:
            r = oracle.cast_ray(w, cam, p, i, j)
            assert r["hash"] == oracle.fnv1a(r["path"].astype("<i4").tobytes())
            assert r["stop_lin"] == (int(r["path"][-1]) if r["steps"] else -1)


# --------------------------------------------- P1/P2: uniform maps ---------

def _random_rays(rng, n, count, margin=3.0):
    O = rng.uniform(-margin, n + margin, size=(count, 3)).astype(np.float32)
    E = rng.uniform(-margin, n + margin, size=(count, 3)).astype(np.float32)
    return O, E


def _pose_from_segment(O, E):
    """Pose with W=H=1, range 1, voxel 1, origin 0: the ray runs O -> O + (E-O)."""
    d = (E - O).astype(np.float32)
    return _axis_pose(O, d), d


def test_all_unknown_steps_identity(oracle_lib):
    """P = 0.5 everywhere: g_R counts the visited voxels, and a 6-connected walk of
    k steps satisfies steps = 1 + sum_a |last_a - first_a|."""
    n = 10
    s = _scene(np.full((n, n, n), 0.5))
    rng = np.random.default_rng(1)
    O, E = _random_rays(rng, n, 400)
    checked = 0
    for o, e in zip(O, E):
        pose, _ = _pose_from_segment(o, e)
        r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
        if r["steps"] == 0:
            assert r["reason"] == oracle.RAY_MISS and r["gain"] == 0.0
            continue
        checked += 1
        assert r["gain"] == float(r["steps"])
        first = np.array(_lin_to_xyz(int(r["path"][0]), n, n))
        last = np.array(_lin_to_xyz(int(r["path"][-1]), n, n))
        assert r["steps"] == 1 + int(np.abs(last - first).sum())
    assert checked > 100


def test_all_free_gain_is_steps_times_p(oracle_lib):
    n = 9
    s = _scene(np.full((n, n, n), 0.2))
    rng = np.random.default_rng(2)
    O, E = _random_rays(rng, n, 300)
    for o, e in zip(O, E):
        pose, _ = _pose_from_segment(o, e)
        r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
        assert r["gain"] == r["steps"] * float(F32(0.2))


def test_axis_aligned_closed_form(oracle_lib):
    """A ray along +x visits floor(E_x) - floor(O_x) + 1 voxels after clipping to [0, n)."""
    n = 16
    s = _scene(np.full((n, n, n), 0.5))
    rng = np.random.default_rng(3)
    for _ in range(300):
        o = rng.uniform(-4, n + 4, size=3).astype(np.float32)
        o[1:] = rng.uniform(0.01, n - 0.01, size=2)
        length = F32(rng.uniform(0.1, 2 * n))
        ex = F32(o[0] + length)
        if min(abs(ex - round(ex)), abs(o[0] - round(o[0]))) < 1e-3:
            continue
        pose = _axis_pose(o, (length, 0.0, 0.0))
        r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
        lo = max(math.floor(o[0]), 0)
        hi = min(math.floor(ex), n - 1)
        expected = hi - lo + 1 if (ex > 0 and o[0] < n) else 0
        assert r["steps"] == max(expected, 0), (o, ex)
        if expected > 0:
            x, y, z = _lin_to_xyz(int(r["path"][-1]), n, n)
            assert (x, y, z) == (hi, math.floor(o[1]), math.floor(o[2]))
            assert r["reason"] == (oracle.RAY_END if ex < n else oracle.RAY_EXIT)


def test_parallel_ray_beside_map_misses(oracle_lib):
    n = 6
    s = _scene(np.full((n, n, n), 0.5))
    pose = _axis_pose((1.5, -0.5, 2.5), (4.0, 0.0, 0.0))       # y = -0.5 is outside
    r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
    assert r["steps"] == 0 and r["reason"] == oracle.RAY_MISS and r["stop_lin"] == -1


def test_nonfinite_pose_is_invalid(oracle_lib):
    s = _scene(np.full((4, 4, 4), 0.5))
    pose = _axis_pose((1.5, 1.5, 1.5), (1.0, 0.0, 0.0))
    pose[0] = np.nan
    r = oracle.cast_ray(s, (3, 3, 0.2, 0.2, 1.0), pose, 1, 1)
    assert r["reason"] == oracle.RAY_INVALID and r["steps"] == 0 and math.isnan(r["gain"])
    ig, _ = oracle.eval_viewpoints(s, (3, 3, 0.2, 0.2, 1.0), pose[None])
    assert math.isnan(float(ig[0]))


# ------------------------------------------------ P3: occupied slab --------

def test_single_occupied_slab(oracle_lib):
    """Free space with one occupied plane x = x0: every ray from x < x0 that reaches the
    plane inside the map stops there, in the voxel holding the exact crossing point."""
    n, x0 = 14, 9
    P = np.full((n, n, n), 0.2, dtype=np.float32)
    P[:, :, x0] = 0.9
    s = _scene(P)
    rng = np.random.default_rng(4)
    hits = 0
    for _ in range(600):
        o = rng.uniform(0.0, x0 - 0.5, size=3).astype(np.float32)
        o[1:] = rng.uniform(0, n, size=2)
        e = rng.uniform(0, n, size=3).astype(np.float32)
        e[0] = rng.uniform(x0 + 1.2, n + 3)
        pose, d = _pose_from_segment(o, e)
        D = [Fraction(float(v)) for v in d]
        Of = [Fraction(float(v)) for v in o]
        tx = (Fraction(x0) - Of[0]) / D[0]
        y = Of[1] + tx * D[1]
        z = Of[2] + tx * D[2]
        if not (0 <= y < n and 0 <= z < n):
            continue
        if min(abs(y - round(y)), abs(z - round(z))) < Fraction(1, 100):
            continue     # crossing near a voxel edge: a tie, not checked
        r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
        assert r["reason"] == oracle.RAY_HIT
        assert _lin_to_xyz(r["stop_lin"], n, n) == (x0, math.floor(y), math.floor(z))
        assert r["gain"] == (r["steps"] - 1) * float(F32(0.2)) + float(F32(1) - F32(0.9))
        hits += 1
    assert hits > 200


# ------------------------------------------------ P4: spheres --------------

def _dist_point_segment(c, a, b):
    ab = b - a
    t = np.clip(np.dot(c - a, ab) / np.dot(ab, ab), 0.0, 1.0)
    return float(np.linalg.norm(a + t * ab - c))


def test_solid_ball_must_and_must_not_hit(oracle_lib):
    n, R = 24, 5.0
    cen = np.array([12.3, 11.7, 12.1])
    idx = np.indices((n, n, n))[::-1].transpose(1, 2, 3, 0) + 0.5
    inside = np.linalg.norm(idx - cen, axis=-1) <= R
    P = np.where(inside, 0.9, 0.5).astype(np.float32)
    s = _scene(P)
    rng = np.random.default_rng(5)
    must, mustnot = 0, 0
    for _ in range(800):
        o = rng.uniform(0, n, size=3).astype(np.float32)
        if np.linalg.norm(o - cen) < R + 1.5:
            continue
        if rng.uniform() < 0.5:
            e = (o + rng.normal(size=3) * 12).astype(np.float32)
        else:
            target = cen + rng.normal(size=3) * 3.0
            e = (o + 2.0 * (target - o)).astype(np.float32)
        pose, d = _pose_from_segment(o, e)
        a = o.astype(np.float64)
        b = a + d.astype(np.float64)
        # clip the segment to the map box before measuring its distance to the centre
        lo, hi = 0.0, 1.0
        for k in range(3):
            if d[k] != 0:
                ta, tb = (0 - a[k]) / d[k], (n - a[k]) / d[k]
                lo, hi = max(lo, min(ta, tb)), min(hi, max(ta, tb))
        if lo >= hi:
            continue
        dist = _dist_point_segment(cen, a + lo * (b - a), a + hi * (b - a))
        r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
        if dist < R - math.sqrt(3) / 2 - 0.01:
            assert r["reason"] == oracle.RAY_HIT
            must += 1
        elif dist > R + math.sqrt(3) / 2 + 0.01:
            assert r["reason"] != oracle.RAY_HIT
            mustnot += 1
    assert must > 50 and mustnot > 50


def test_hollow_shell_from_centre(oracle_lib):
    """Camera at the centre of a 2-voxel-thick shell: every ray hits the shell, after
    a number of steps bracketed by the ray's L1 length to the shell."""
    n = 32
    cen = np.array([16.0, 16.0, 16.0], dtype=np.float32)
    r_in, r_out = 9.0, 11.0
    idx = np.indices((n, n, n))[::-1].transpose(1, 2, 3, 0) + 0.5
    dist = np.linalg.norm(idx - cen, axis=-1)
    P = np.where((dist >= r_in) & (dist <= r_out), 0.9, 0.2).astype(np.float32)
    s = _scene(P)
    cam = Camera(17, 13, 70, 55, 14.0)
    rng = np.random.default_rng(6)
    dirs = rng.normal(size=(6, 3))
    poses = look_at(np.repeat(cen[None].astype(np.float64), 6, 0), cen + dirs)
    lmin, lmax = r_in - math.sqrt(3) / 2, r_out + math.sqrt(3) / 2
    dh = F32(F32(14.0) * cam.tan_h)
    dv = F32(F32(14.0) * cam.tan_v)
    for p in poses:
        R = p[:9].astype(np.float64).reshape(3, 3)
        for j in range(cam.height):
            for i in range(cam.width):
                u = float(dh) * (2 * i - (cam.width - 1)) / (cam.width - 1)
                v = float(dv) * (2 * j - (cam.height - 1)) / (cam.height - 1)
                dvec = R @ np.array([u, v, 14.0])
                dhat = dvec / np.linalg.norm(dvec)
                r = oracle.cast_ray(s, cam, p, i, j)
                assert r["reason"] == oracle.RAY_HIT
                l1 = np.abs(dhat).sum()
                assert lmin * l1 - 2 <= r["steps"] <= lmax * l1 + 4


# ------------------------------------------------ P5: exact brute force -----

def _exact_walk(O, D, n):
    """Voxels whose interior the segment O + t*D, t in [0,1], crosses (exact rationals).

    Returns (sequence, near_tie) where near_tie marks rays with two plane
    crossings, or a crossing and the endpoint, closer than 1e-5 in t.
    """
    Of = [Fraction(float(v)) for v in O]
    Df = [Fraction(float(v)) for v in D]
    t0, t1 = Fraction(0), Fraction(1)
    for a in range(3):
        if Df[a] == 0:
            if not (0 <= Of[a] < n):
                return [], False
            continue
        ta = (0 - Of[a]) / Df[a]
        tb = (n - Of[a]) / Df[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    if t0 >= t1:
        return [], t0 == t1
    crossings = []
    for a in range(3):
        if Df[a] == 0:
            continue
        lo = Of[a] + t0 * Df[a]
        hi = Of[a] + t1 * Df[a]
        kmin, kmax = (lo, hi) if lo <= hi else (hi, lo)
        for k in range(max(1, math.floor(kmin)), min(n - 1, math.ceil(kmax)) + 1):
            t = (k - Of[a]) / Df[a]
            if t0 < t < t1:
                crossings.append((t, a))
    crossings.sort()
    eps = Fraction(1, 100000)
    near = False
    times = [t0] + [c[0] for c in crossings] + [t1]
    for k in range(1, len(times)):
        if times[k] - times[k - 1] < eps:
            near = True
    first_t = (t0 + (crossings[0][0] if crossings else t1)) / 2
    cur = [math.floor(Of[a] + first_t * Df[a]) for a in range(3)]
    seq = [tuple(cur)]
    for t, a in crossings:
        cur[a] += 1 if Df[a] > 0 else -1
        seq.append(tuple(cur))
    return seq, near


def test_bruteforce_exact_walk(oracle_lib):
    rng = np.random.default_rng(7)
    exact_ok, near_ties = 0, 0
    for n in (3, 7, 12):
        s = _scene(np.full((n, n, n), 0.2))
        O, E = _random_rays(rng, n, 250)
        for o, e in zip(O, E):
            pose, d = _pose_from_segment(o, e)
            r = oracle.cast_ray(s, (1, 1, 0.1, 0.1, 1.0), pose, 0, 0)
            got = [_lin_to_xyz(int(v), n, n) for v in r["path"]]
            seq, near = _exact_walk(o, d, n)
            # P6: a 6-connected walk, one axis changes by one per step
            for a_, b_ in zip(got, got[1:]):
                assert sum(abs(x - y) for x, y in zip(a_, b_)) == 1
            # sampled points of the clipped segment, away from voxel faces, lie in visited voxels
            ts = rng.uniform(0, 1, 200)
            pts = o[None].astype(np.float64) + ts[:, None] * d[None].astype(np.float64)
            inb = np.all((pts >= 0) & (pts < n), axis=1)
            frac = np.abs(pts - np.round(pts))
            safe = inb & np.all(frac > 1e-3, axis=1)
            gotset = set(got)
            for pnt in pts[safe]:
                assert tuple(int(v) for v in np.floor(pnt)) in gotset
            if near:
                near_ties += 1
                continue
            assert got == seq, (o, e)
            exact_ok += 1
    assert exact_ok > 600 and near_ties < 30


# ------------------------------------------------ P6: invariants -----------

def test_no_occupied_voxel_before_stop_and_permutation(oracle_lib):
    sc = scene_spheres(n=32, voxel=0.1, n_spheres=12, seed=11)
    cam = Camera(11, 9, 60, 45, 2.0)
    poses = poses_sphere(sc.poi, 0.8, 6, seed=12)
    d = oracle.trace_rays(sc, cam, poses)
    flatP = sc.P.ravel()
    for p in range(2):
        for k in range(0, cam.rays, 7):
            r = oracle.cast_ray(sc, cam, poses[p], k % cam.width, k // cam.width)
            assert np.all(flatP[r["path"][:-1]] <= 0.5)
            assert r["hash"] == d["hash"][p, k] and r["steps"] == d["steps"][p, k]
    ig, st = oracle.eval_viewpoints(sc, cam, poses)
    perm = np.array([3, 0, 5, 1, 4, 2])
    ig2, st2 = oracle.eval_viewpoints(sc, cam, poses[perm])
    assert np.array_equal(ig[perm], ig2) and np.array_equal(st[perm], st2)
    ig3, _ = oracle.eval_viewpoints(sc, cam, poses)
    assert np.array_equal(ig, ig3)
    # the per-perspective IG is the mean of its ray gains (mean over N_E rays)
    assert np.allclose(ig, d["gain"].mean(axis=1), rtol=1e-7)
    assert np.array_equal(st, d["steps"].sum(axis=1))


def test_border_rays_reach_far_plane_corners(oracle_lib):
    """The corner rays of the grid end at t + R (+-d_h, +-d_v, d_Cam) (Sec. III endpoints)."""
    n, vox = 64, 0.05
    s = _scene(np.full((n, n, n), 0.5), voxel=vox)
    cam = Camera(5, 4, 60, 45, 1.0)
    rng = np.random.default_rng(13)
    poses = look_at(np.array([[1.1, 1.3, 1.2]]), np.array([1.6, 1.8, 1.5]) + rng.normal(size=3) * 0.1)
    p = poses[0]
    R = p[:9].astype(np.float64).reshape(3, 3)
    dh, dv = 1.0 * float(cam.tan_h), 1.0 * float(cam.tan_v)
    for (i, j, su, sv) in [(0, 0, -1, -1), (4, 0, 1, -1), (0, 3, -1, 1), (4, 3, 1, 1), (2, 0, 0, -1)]:
        e = p[9:].astype(np.float64) + R @ np.array([su * dh, sv * dv, 1.0])
        r = oracle.cast_ray(s, cam, p, i, j)
        assert r["reason"] == oracle.RAY_END
        expect = tuple(int(v) for v in np.floor(e / vox))
        assert _lin_to_xyz(r["stop_lin"], n, n) == expect


# ------------------------------------------------ P7: paper's observation ---

def test_ig_decreases_toward_object(oracle_lib):
    """Perspectives closer to an object see less (Sec. III): on a line toward a
    single occupied ball in unknown space, IG does not increase as the camera approaches."""
    n, vox = 96, 0.05
    idx = (np.indices((n, n, n))[::-1].transpose(1, 2, 3, 0) + 0.5) * vox
    cen = np.array([2.4, 2.4, 2.4])
    P = np.where(np.linalg.norm(idx - cen, axis=-1) <= 0.3, 0.9, 0.5).astype(np.float32)
    s = _scene(P, voxel=vox)
    cam = Camera(24, 18, 60, 45, 1.5)
    dists = np.linspace(1.6, 0.45, 12)
    pos = cen[None] + dists[:, None] * np.array([[0.6, -0.48, 0.64]])
    ig, _ = oracle.eval_viewpoints(s, cam, look_at(pos, cen))
    assert np.all(np.diff(ig) <= 1e-3 * ig[:-1])
    assert ig[-1] < 0.6 * ig[0]


# ------------------------------------------------ P8: trajectory union -----

def _traj_scene():
    sc = scene_spheres(n=40, voxel=0.1, n_spheres=15, seed=21)
    cam = Camera(10, 8, 60, 45, 1.8)
    return sc, cam


def test_trajectory_union_matches_distinct_voxels(oracle_lib):
    """|U| and the class counts equal those of the distinct voxels over the full ray
    paths of all poses; visits equal the summed per-perspective steps."""
    from workloads import trajectories_walk
    sc, cam = _traj_scene()
    traj = trajectories_walk(sc.poi, 3, 4, seed=22)
    ig, counts, visits = oracle.eval_trajectories(sc, cam, traj)
    flatP = sc.P.ravel()
    for t in range(traj.shape[0]):
        seen = set()
        per_pose = []
        for l in range(traj.shape[1]):
            mine = set()
            for j in range(cam.height):
                for i in range(cam.width):
                    mine.update(int(v) for v in oracle.cast_ray(sc, cam, traj[t, l], i, j)["path"])
            per_pose.append(len(mine))
            seen |= mine
        vals = flatP[np.array(sorted(seen))]
        assert counts[t, 0] == len(seen)
        assert counts[t, 1] == np.count_nonzero(vals > 0.5)
        assert counts[t, 2] == np.count_nonzero(vals < 0.5)
        assert counts[t, 3] == np.count_nonzero(vals == 0.5)
        assert counts[t, 0] <= sum(per_pose)
        g = np.where(vals > 0.5, np.float32(1) - vals, np.where(vals < 0.5, vals, np.float32(1)))
        assert ig[t] == pytest.approx(float(np.sum(g.astype(np.float64))), rel=1e-7)
        _, st = oracle.eval_viewpoints(sc, cam, traj[t])
        assert visits[t] == st.sum()


def test_trajectory_duplicate_and_permutation_invariance(oracle_lib):
    from workloads import trajectories_walk
    sc, cam = _traj_scene()
    traj = trajectories_walk(sc.poi, 2, 5, seed=23)
    ig, counts, visits = oracle.eval_trajectories(sc, cam, traj)
    perm = traj[:, [4, 2, 0, 3, 1]]
    ig2, counts2, _ = oracle.eval_trajectories(sc, cam, perm)
    assert np.array_equal(counts, counts2) and np.array_equal(ig, ig2)
    dup = np.concatenate([traj, traj[:, :2]], axis=1)
    ig3, counts3, visits3 = oracle.eval_trajectories(sc, cam, dup)
    assert np.array_equal(counts, counts3) and np.array_equal(ig, ig3)
    assert np.all(visits3 > visits)
