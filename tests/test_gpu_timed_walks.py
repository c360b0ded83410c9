"""Per-ray parity of the walks that the throughput kernels run (through the C ABI).

nbt_ig_trace_viewpoints and nbt_ig_trace_trajectories run the same kernels as
nbt_ig_eval_viewpoints and nbt_ig_eval_trajectories -- pipelined gathers,
incremental byte offsets in the map's storage order, sentinel refills, the
union walk's bitset marks -- instantiated to also write one record per ray,
built from the offsets the walk gathered (decoded back into voxel
coordinates).  Bar (Sec. III, IG calculation: the ray's voxels up to and
including the first occupied one or the endpoint): every record's step count,
stop voxel, stop reason and FNV-1a-64 of the visited linear indices equal the
oracle's bit for bit, its binary64 gain too (same summation order); for the
union walk no visit's bitset position names another voxel than the one
gathered; the kernels' IG, step, count and visit outputs are the bits of the
untraced calls.  Every test runs once per map storage order.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import look_at, make_config, poses_sphere, scene_spheres, trajectories_walk
from workloads.configs import Camera
from workloads.scenes import SceneMap

pytestmark = pytest.mark.gpu

IG_RTOL = 1e-5


def _note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nbt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_22588_amd as nbt
    return nbt


@pytest.fixture(scope="module", params=[0, 1, 2, 3], ids=["linear", "column4", "column2", "column8"])
def ctx(nbt, request):
    c = nbt.Context(0)
    c.set_map_layout(request.param)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _records_equal(d, ref, what):
    """Records (dict of tensors, any leading shape) against the oracle's (flattened rays)."""
    for key in ("steps", "stop_lin", "reason"):
        got = d[key].cpu().numpy().reshape(-1).astype(np.int64)
        exp = ref[key].reshape(-1).astype(np.int64)
        bad = np.flatnonzero(got != exp)
        assert bad.size == 0, f"{what}: {key} differs at rays {bad[:5].tolist()}: got {got[bad[0]]} want {exp[bad[0]]}"
    h = d["hash"].cpu().numpy().reshape(-1).view(np.uint64)
    bad = np.flatnonzero(h != ref["hash"].reshape(-1))
    assert bad.size == 0, f"{what}: voxel sequence hash differs at rays {bad[:5].tolist()}"
    g = d["gain"].cpu().numpy().reshape(-1)
    rg = ref["gain"].reshape(-1)
    ok = (g.view(np.uint64) == rg.view(np.uint64)) | (np.isnan(g) & np.isnan(rg))
    assert ok.all(), f"{what}: ray gain differs at rays {np.flatnonzero(~ok)[:5].tolist()}"


def _ig_rel(ig, ref):
    ig = np.asarray(ig, np.float64)
    ref = np.asarray(ref, np.float64)
    assert np.array_equal(np.isnan(ig), np.isnan(ref))
    ok = ~np.isnan(ref)
    rel = np.abs(ig[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), 1e-30)
    return float(rel.max()) if rel.size else 0.0


def _launch(ctx, waves=4, tw=3, tpw=0, remap=0, depth=8):
    ctx.set_launch(waves, tw, tpw, remap, depth)


# shapes: (waves, tile_w_log2, tiles_per_wave, xcd_remap, depth); the first is the default
SHAPES = [(4, 3, 0, 0, 8), (4, 3, 0, 0, 4), (4, 3, 0, 0, 2), (2, 2, 3, 1, 8), (8, 4, 1, 0, 4), (1, 3, 2, 0, 1),
          (1, 3, 4, 0, 8)]


def _trace_vp(nbt, m, cam, dposes, want_steps):
    import torch
    ig, st, d = nbt.trace_viewpoints(m, cam, dposes, want_steps=want_steps)
    ig0, st0 = nbt.eval_viewpoints(m, cam, dposes, want_steps=want_steps)
    torch.cuda.synchronize()
    # the parity instance leaves the kernel's own outputs unchanged
    assert np.array_equal(ig.cpu().numpy().view(np.uint32), ig0.cpu().numpy().view(np.uint32))
    if want_steps:
        assert np.array_equal(st.cpu().numpy(), st0.cpu().numpy())
    assert np.all(d["reserved"].cpu().numpy() == 0)
    return ig, st, d


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "w{}t{}p{}x{}d{}".format(*s))
def test_cfg1_timed_walk_every_ray(nbt, ctx, shape):
    """Config 1, all 32 perspectives x 3072 rays, in several launch shapes and pipeline
    depths, with and without the visit count."""
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note(f"cfg1 timed walk, shape {shape}")
    m = nbt.Map(ctx, scene.P, scene.voxel, scene.origin)
    ref = oracle.trace_rays(scene, cam, poses)
    ig_ref, st_ref = oracle.eval_viewpoints(scene, cam, poses)
    dp = _dev(poses)
    _launch(ctx, *shape)
    try:
        for want_steps in (True, False):
            ig, st, d = _trace_vp(nbt, m, cam, dp, want_steps)
            _records_equal(d, ref, f"cfg1 {shape} steps={want_steps}")
            assert _ig_rel(ig.cpu().numpy(), ig_ref) <= IG_RTOL
            if want_steps:
                assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref)
    finally:
        _launch(ctx)
    assert np.count_nonzero(ref["reason"] == oracle.RAY_HIT) > 100
    assert np.count_nonzero(ref["reason"] == oracle.RAY_EXIT) > 100
    m.close()


def test_timed_walk_edge_cases(nbt, ctx):
    """Camera inside an occupied block, rays missing the map, P = 0 and P = 1 voxels,
    1x1 / 1xH / Wx1 grids, a non-finite pose, tiny and flat maps."""
    _note("timed walk edge cases")
    n = 20
    P = np.full((n, n, n), 0.5, dtype=np.float32)
    P[5:8, 5:8, 5:8] = 1.0
    P[10:14, 2:6, 3:9] = 0.0
    P[0, :, :] = 0.9
    P[:, :, 15] = 0.2
    origin = np.array([0.3, -0.2, 0.1], np.float32)
    centre = origin.astype(np.float64) + 1.0
    sc = SceneMap(P=P, voxel=0.1, origin=origin, poi=centre)
    pos = np.array([centre, centre + [0.0, 0.0, 5.0], origin + [0.65, 0.65, 0.65], origin + [-0.5, -0.5, -0.5]])
    poses = look_at(pos, centre)
    away = look_at(centre[None] + [[0.0, 0.0, 5.0]], centre[None] + [[0.0, 0.0, 10.0]])
    nanpose = poses[:1].copy()
    nanpose[0, 4] = np.nan
    allp = np.concatenate([poses, away, nanpose], axis=0)
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    for cam in (Camera(1, 1, 40, 30, 1.5), Camera(1, 9, 40, 30, 1.5), Camera(13, 1, 50, 30, 3.0),
                Camera(29, 17, 90, 70, 0.4)):
        for depth in (8, 2):
            _launch(ctx, depth=depth)
            try:
                _, _, d = _trace_vp(nbt, m, cam, _dev(allp), True)
            finally:
                _launch(ctx)
            _records_equal(d, oracle.trace_rays(sc, cam, allp), f"edge {cam} depth {depth}")
    m.close()
    rng = np.random.default_rng(5)
    for dims in [(1, 1, 1), (7, 1, 1), (1, 5, 9), (3, 4, 2), (9, 10, 11)]:
        nx, ny, nz = dims
        Pt = rng.choice(np.array([0.1, 0.5, 0.95], np.float32), size=(nz, ny, nx))
        c = np.array([nx, ny, nz]) * 0.25
        st = SceneMap(P=Pt, voxel=0.5, origin=np.zeros(3, np.float32), poi=c)
        pz = look_at(c + rng.normal(size=(9, 3)) * 1.5, c + rng.normal(size=3) * 0.2)
        cam = Camera(11, 7, 80, 60, 4.0)
        mt = nbt.Map(ctx, st.P, st.voxel, st.origin)
        _, _, d = _trace_vp(nbt, mt, cam, _dev(pz), False)
        _records_equal(d, oracle.trace_rays(st, cam, pz), f"tiny {dims}")
        mt.close()


def test_cfg2_timed_walk_sampled(nbt, ctx):
    """Config 2 at its real size (256^3 at 2 cm, 160x120 rays, 3 m) in the launch shapes the
    full 4096-perspective call uses (the default's and the two the autotuner picks): every
    ray of 64 seeded perspectives, bit for bit; their IG and step counts also equal the full
    call's bits."""
    import torch
    w = make_config(2)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note(f"cfg2 timed walk: 64 of {poses.shape[0]} perspectives")
    m = nbt.Map(ctx, scene.P, scene.voxel, scene.origin)
    rng = np.random.default_rng(22588)
    pick = np.sort(rng.choice(poses.shape[0], size=64, replace=False))
    ref = oracle.trace_rays(scene, cam, poses[pick])
    ig_ref, st_ref = oracle.eval_viewpoints(scene, cam, poses[pick])
    # 160x120 rays in 8x8 tiles = 300 tiles; the default resolves to 4 waves of 15 tiles per
    # workgroup (5 per perspective) for 4096 perspectives; the tuner picks single waves of 4
    # or 2 tiles (75 or 150 per perspective)
    for shape in ((4, 3, 15, 0, 8), (1, 3, 4, 0, 8), (1, 3, 2, 0, 8)):
        _note(f"cfg2 timed walk, shape {shape}")
        _launch(ctx, *shape)
        try:
            ig_all, st_all = nbt.eval_viewpoints(m, cam, _dev(poses))
            ig, st, d = _trace_vp(nbt, m, cam, _dev(poses[pick]), True)
        finally:
            _launch(ctx)
        torch.cuda.synchronize()
        assert np.array_equal(ig.cpu().numpy().view(np.uint32), ig_all.cpu().numpy()[pick].view(np.uint32))
        assert np.array_equal(st.cpu().numpy(), st_all.cpu().numpy()[pick])
        _records_equal(d, ref, f"cfg2 sample {shape}")
        assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref)
        assert _ig_rel(ig.cpu().numpy(), ig_ref) <= IG_RTOL
    m.close()


def _trace_traj(nbt, m, cam, traj, want_visits=True):
    import torch
    dp = _dev(traj)
    ig, counts, visits, d = nbt.trace_trajectories(m, cam, dp, want_visits=want_visits)
    ig0, counts0, visits0 = nbt.eval_trajectories(m, cam, dp, want_visits=want_visits)
    torch.cuda.synchronize()
    assert np.array_equal(ig.cpu().numpy().view(np.uint32), ig0.cpu().numpy().view(np.uint32))
    assert np.array_equal(counts.cpu().numpy(), counts0.cpu().numpy())
    if want_visits:
        assert np.array_equal(visits.cpu().numpy(), visits0.cpu().numpy())
    mism = d["reserved"].cpu().numpy()
    assert np.all(mism == 0), f"{int((mism != 0).sum())} rays marked a voxel other than the one gathered"
    return ig, counts, visits, d


def _traj_ref_check(sc, cam, traj, got, d, what):
    ig, counts, visits = got
    T, L = traj.shape[:2]
    ref = oracle.trace_rays(sc, cam, traj.reshape(T * L, 12))
    _records_equal(d, ref, what)
    ig_ref, counts_ref, visits_ref = oracle.eval_trajectories(sc, cam, traj)
    assert np.array_equal(counts.cpu().numpy().astype(np.uint32), counts_ref), what
    if visits is not None:
        assert np.array_equal(visits.cpu().numpy().view(np.uint64), visits_ref), what
    assert _ig_rel(ig.cpu().numpy(), ig_ref) <= IG_RTOL, what


def test_union_walk_every_ray(nbt, ctx):
    """The trajectory union walk on 10 trajectories x 5 poses x 41x29 rays: every ray's record
    and every mark, for each workgroup size, with and without the visit count, in one LDS
    pass and in several (LDS budgets that split each box into 2..40 slices)."""
    sc = scene_spheres(n=(64, 56, 60), voxel=0.05, n_spheres=40, seed=401, origin=(0.1, -0.3, 0.2))
    cam = Camera(41, 29, 60, 45, 1.2)
    traj = trajectories_walk(sc.poi, 10, 5, seed=402)
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    _note("union walk records")
    try:
        for waves in (8, 4, 16):
            ctx.set_traj_waves(waves)
            for budget in (0, 8 * 1024, 1024):
                ctx.set_lds_budget(budget)
                for want_visits in (True, False):
                    ig, counts, visits, d = _trace_traj(nbt, m, cam, traj, want_visits)
                    _traj_ref_check(sc, cam, traj, (ig, counts, visits), d,
                                    f"waves {waves} budget {budget} visits {want_visits}")
    finally:
        ctx.set_traj_waves(8)
        ctx.set_lds_budget(0)
    m.close()


def test_cfg4_union_walk_sampled(nbt, ctx):
    """Config 4 at its real size (256^3 at 5 cm, 24 poses x 128x96 rays per trajectory): all
    4096 trajectories on the GPU; 8 seeded trajectories, with the largest box among them,
    traced ray by ray in the same launch and checked against the oracle."""
    import torch
    w = make_config(4)
    sc, cam, traj = w.maps[0], w.camera, w.poses[0]
    _note(f"cfg4 union walk: 8 of {traj.shape[0]} trajectories")
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    ig_all, counts_all, visits_all = nbt.eval_trajectories(m, cam, _dev(traj))
    torch.cuda.synchronize()
    counts_all = counts_all.cpu().numpy()
    rng = np.random.default_rng(4096)
    pick = np.sort(np.unique(np.concatenate([rng.choice(traj.shape[0], size=7, replace=False),
                                             [int(np.argmax(counts_all[:, 0]))]])))
    ig, counts, visits, d = _trace_traj(nbt, m, cam, traj[pick])
    assert np.array_equal(ig.cpu().numpy().view(np.uint32), ig_all.cpu().numpy()[pick].view(np.uint32))
    assert np.array_equal(counts.cpu().numpy(), counts_all[pick])
    assert np.array_equal(visits.cpu().numpy(), visits_all.cpu().numpy()[pick])
    _traj_ref_check(sc, cam, traj[pick], (ig, counts, visits), d, "cfg4 sample")
    m.close()


def test_whole_map_union_passes(nbt, ctx):
    """Tiny maps seen whole from every pose (each box is the whole map, nx*ny*nz bits on and
    beside multiples of 32): records and marks in one pass, at the exact fit of the box and
    one word under it (two passes), and the results' bits independent of the pass count."""
    _note("whole-map boxes, passes")
    for shape in [(31, 1, 1), (11, 3, 1), (16, 4, 2), (9, 7, 5)]:
        nx, ny, nz = shape
        rng = np.random.default_rng(4100 + 97 * nx + 13 * ny + nz)
        P = rng.choice(np.array([0.05, 0.2, 0.35, 0.5, 0.9], np.float32), size=(nz, ny, nx),
                       p=[0.1, 0.3, 0.15, 0.4, 0.05])
        origin = np.array([0.3, -0.2, 0.1], np.float32)
        centre = origin.astype(np.float64) + 0.05 * np.array([nx, ny, nz], np.float64)
        sc = SceneMap(P=P, voxel=0.1, origin=origin, poi=centre)
        cam = Camera(23, 17, 100.0, 90.0, 8.0)
        dd = rng.normal(size=(12, 3))
        dd /= np.linalg.norm(dd, axis=1, keepdims=True)
        traj = look_at(centre + 2.5 * dd, centre).reshape(3, 4, 12)
        m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
        nbits = nx * ny * nz
        fit = (-(-nbits // 32) + 2) * 4
        outs = []
        try:
            for budget in (0, fit, fit - 4, 12):
                ctx.set_lds_budget(budget)
                ig, counts, visits, d = _trace_traj(nbt, m, cam, traj)
                _traj_ref_check(sc, cam, traj, (ig, counts, visits), d, f"{shape} budget {budget}")
                outs.append((ig.cpu().numpy().view(np.uint32), counts.cpu().numpy()))
        finally:
            ctx.set_lds_budget(0)
        for o in outs[1:]:
            assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1]), shape
        m.close()


def test_depths_give_the_same_bits(nbt, ctx):
    """The IG-only walk sums gains in binary32 runs of 8 slots at fixed slot indices, so
    pipeline depths 2, 4 and 8 give the same IG bits (same workgroup shape)."""
    import torch
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note("timed walk: IG bits across pipeline depths")
    m = nbt.Map(ctx, scene.P, scene.voxel, scene.origin)
    dp = _dev(poses)
    got = {}
    try:
        for depth in (2, 4, 8):
            _launch(ctx, depth=depth)
            ig, _ = nbt.eval_viewpoints(m, cam, dp, want_steps=False)
            torch.cuda.synchronize()
            got[depth] = ig.cpu().numpy().view(np.uint32)
    finally:
        _launch(ctx)
    for depth in (2, 4):
        assert np.array_equal(got[depth], got[8]), depth
    m.close()
