"""GPU parity of the per-trajectory union IG against the CPU oracle (through the C ABI).

Bar: |U|, per-state counts and total visits bit-exact; union IG within 1e-5
relative.  Boxes that fit the LDS slice in one pass and boxes covered in
several passes are both exercised.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from workloads import look_at, make_config, scene_spheres, trajectories_walk
from workloads.configs import Camera
from workloads.scenes import SceneMap

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def nbt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_22588_amd as nbt
    return nbt


@pytest.fixture(scope="module", params=[0, 1, 2, 3], ids=["linear", "column4", "column2", "column8"])
def ctx(nbt, request):
    """Every test of this module runs once per map layout."""
    c = nbt.Context(0)
    c.set_map_layout(request.param)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(nbt, m, cam, traj):
    import torch
    ig, counts, visits = nbt.eval_trajectories(m, cam, _dev(traj))
    torch.cuda.synchronize()
    return ig.cpu().numpy(), counts.cpu().numpy().astype(np.uint32), visits.cpu().numpy().view(np.uint64)


def _check(got, ref):
    ig, counts, visits = got
    ig_ref, counts_ref, visits_ref = ref
    assert np.array_equal(counts, counts_ref), (np.argwhere(counts != counts_ref)[:5], counts[:3], counts_ref[:3])
    assert np.array_equal(visits, visits_ref)
    nan = np.isnan(ig_ref)
    assert np.array_equal(np.isnan(ig), nan)
    rel = np.abs(ig[~nan] - ig_ref[~nan]) / np.maximum(np.abs(ig_ref[~nan]), 1e-30)
    assert rel.size == 0 or rel.max() <= 1e-5, rel.max()


@pytest.fixture(scope="module")
def small(nbt, ctx):
    sc = scene_spheres(n=(64, 56, 60), voxel=0.05, n_spheres=40, seed=401, origin=(0.1, -0.3, 0.2))
    cam = Camera(41, 29, 60, 45, 1.2)
    traj = trajectories_walk(sc.poi, 10, 5, seed=402)
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    ref = oracle.eval_trajectories(sc, cam, traj)
    return sc, cam, traj, m, ref


def test_small_lds_path(nbt, ctx, small):
    sc, cam, traj, m, ref = small
    _note(f"trajectories: LDS path, context {ctx.info()}")
    ctx.set_lds_budget(0)
    assert ctx.get_traj_waves() == 8
    try:
        for waves in (8, 4, 16):                  # workgroup size does not change the result
            ctx.set_traj_waves(waves)
            _check(_run(nbt, m, cam, traj), ref)
    finally:
        ctx.set_traj_waves(8)
    with pytest.raises(nbt.NbtError):
        ctx.set_traj_waves(6)
    assert ref[1][:, 0].min() > 1000
    # without visits the walk keeps no count; IG and counts are the same bits
    import torch
    ig, counts, visits = nbt.eval_trajectories(m, cam, _dev(traj), want_visits=False)
    torch.cuda.synchronize()
    assert visits is None
    got = _run(nbt, m, cam, traj)
    assert np.array_equal(ig.cpu().numpy().view(np.uint32), got[0].view(np.uint32))
    assert np.array_equal(counts.cpu().numpy().astype(np.uint32), got[1])


def test_small_multi_pass(nbt, ctx, small):
    sc, cam, traj, m, ref = small
    _note("trajectories: several LDS passes per box")
    base = _run(nbt, m, cam, traj)
    try:
        ctx.set_lds_budget(64)                # 14 words per pass: every box takes many passes
        got = _run(nbt, m, cam, traj)
        _check(got, ref)
        assert np.array_equal(got[0].view(np.uint32), base[0].view(np.uint32))
        ctx.set_lds_budget(30 * 1024)         # some boxes fit one pass, some take two
        _check(_run(nbt, m, cam, traj), ref)
        ig, counts, _ = nbt.eval_trajectories(m, cam, _dev(traj), want_visits=False)
        assert np.array_equal(counts.cpu().numpy().astype(np.uint32), ref[1])
        ctx.set_traj_waves(4)
        _check(_run(nbt, m, cam, traj), ref)
    finally:
        ctx.set_lds_budget(0)
        ctx.set_traj_waves(8)


def test_autotune_trajectories(nbt, ctx, small):
    sc, cam, traj, _, ref = small
    _note("trajectories: autotuner")
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    try:
        lay, waves, ms = nbt.autotune_trajectories(m, cam, _dev(traj))
        assert lay in (0, 1, 2, 3) and waves in (4, 8, 16) and ms > 0
        assert m.info()["layout"] == lay and ctx.get_traj_waves() == waves
        _check(_run(nbt, m, cam, traj), ref)
        with pytest.raises(nbt.NbtError):
            nbt.autotune_trajectories(m, cam, _dev(traj[:0]))
    finally:
        ctx.set_traj_waves(8)
        m.close()


def test_single_pose_equals_distinct_voxels(nbt, ctx, small):
    import torch
    sc, cam, traj, m, _ = small
    one = traj[:3, :1]
    ig, counts, visits = _run(nbt, m, cam, one)
    d = nbt.trace_rays(m, cam, _dev(one[:, 0]))
    torch.cuda.synchronize()
    for t in range(3):
        paths = set()
        for k in range(cam.rays):
            paths.update(int(v) for v in oracle.cast_ray(sc, cam, one[t, 0], k % cam.width, k // cam.width)["path"])
        assert counts[t, 0] == len(paths)
        assert visits[t] == int(d["steps"][t].sum().item())


def test_duplicates_and_permutation(nbt, ctx, small):
    sc, cam, traj, m, _ = small
    base = _run(nbt, m, cam, traj)
    perm = _run(nbt, m, cam, traj[:, ::-1].copy())
    dup = _run(nbt, m, cam, np.concatenate([traj, traj[:, :2]], axis=1))
    assert np.array_equal(base[1], perm[1]) and np.array_equal(base[1], dup[1])
    assert np.array_equal(base[0], perm[0]) and np.array_equal(base[0], dup[0])
    assert np.all(dup[2] > base[2])


def test_edge_cases(nbt, ctx, small):
    import torch
    sc, cam, traj, m, _ = small
    _note("trajectories: edge cases")
    bad = traj[:3].copy()
    bad[1, 2, 0] = np.inf
    out = _run(nbt, m, cam, bad)
    ref = oracle.eval_trajectories(sc, cam, bad)
    _check(out, ref)
    assert math.isnan(out[0][1]) and not math.isnan(out[0][0])
    # empty trajectories (no poses) and a no-op call
    empty = np.zeros((2, 0, 12), np.float32)
    ig, counts, visits = nbt.eval_trajectories(m, cam, torch.zeros((2, 0, 12), device="cuda"))
    torch.cuda.synchronize()
    assert np.all(counts.cpu().numpy() == 0) and np.all(ig.cpu().numpy() == 0) and np.all(visits.cpu().numpy() == 0)
    ig, counts, visits = nbt.eval_trajectories(m, cam, torch.zeros((0, 4, 12), device="cuda"))
    assert ig.numel() == 0
    # a trajectory that looks away from the map sees nothing
    away = look_at(np.array([[-5.0, -5.0, -5.0]] * 2), np.array([-9.0, -9.0, -9.0]))[None]
    out = _run(nbt, m, cam, away)
    assert np.all(out[1] == 0) and out[0][0] == 0.0


@pytest.mark.parametrize("shape", [(31, 1, 1), (8, 4, 1), (11, 3, 1), (4, 4, 4), (16, 4, 2), (9, 7, 5)],
                         ids=lambda s: "x".join(map(str, s)))
def test_whole_map_boxes(nbt, ctx, shape):
    """Tiny maps seen whole from every pose: each trajectory's box is the whole map, so its
    bitset has nx*ny*nz bits, on and beside multiples of 32 (the last word of an LDS bitset and
    the bit that out-of-box indices are clamped to).  Also the LDS budget at the exact fit of
    the box, one word under it (two passes) and the default."""
    nx, ny, nz = shape
    _note(f"trajectories: whole-map boxes {shape}")
    rng = np.random.default_rng(4100 + 97 * nx + 13 * ny + nz)
    P = rng.choice(np.array([0.05, 0.2, 0.35, 0.5, 0.9], np.float32), size=(nz, ny, nx),
                   p=[0.1, 0.3, 0.15, 0.4, 0.05])
    voxel = 0.1
    origin = np.array([0.3, -0.2, 0.1], np.float32)
    centre = origin.astype(np.float64) + 0.5 * voxel * np.array([nx, ny, nz], np.float64)
    sc = SceneMap(P=P, voxel=voxel, origin=origin, poi=centre)
    cam = Camera(23, 17, 100.0, 90.0, 8.0)
    d = rng.normal(size=(12, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    traj = look_at(centre + 2.5 * d, centre).reshape(3, 4, 12)
    ref = oracle.eval_trajectories(sc, cam, traj)
    assert np.all(ref[1][:, 0] > 0)
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    nbits = nx * ny * nz
    fit = (-(-nbits // 32) + 2) * 4    # ceil(nbits / 32) words, room for the clamp bit, the all-ones word
    try:
        for budget in (0, fit, fit - 4):
            ctx.set_lds_budget(budget)
            _check(_run(nbt, m, cam, traj), ref)
    finally:
        ctx.set_lds_budget(0)


def test_cfg4_full_size_sampled(nbt, ctx):
    """Config 4 at its real size (4096 trajectories x 24 poses x 128x96 rays on a 256^3 map):
    all trajectories on the GPU, the oracle on 8 seeded trajectories."""
    w = make_config(4)
    sc, cam, traj = w.maps[0], w.camera, w.poses[0]
    _note(f"cfg4 full size: {traj.shape}")
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    ig, counts, visits = _run(nbt, m, cam, traj)
    rng = np.random.default_rng(44)
    pick = np.sort(rng.choice(traj.shape[0], size=8, replace=False))
    ref = oracle.eval_trajectories(sc, cam, traj[pick])
    _check((ig[pick], counts[pick], visits[pick]), ref)
    assert np.all(counts[:, 0] == counts[:, 1:].sum(axis=1))
    assert np.all(counts[:, 0] > 0)
