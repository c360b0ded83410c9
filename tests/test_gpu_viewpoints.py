"""GPU parity of the per-perspective IG path against the CPU oracle (through the C ABI).

Bar: voxel walks bit-exact (per-ray step count, stop voxel, stop reason and
FNV-1a digest of the visited linear indices), per-perspective voxel-step
totals exact, IG within 1e-5 relative (float32 result of a float64 sum).
"""

import math
import sys

import numpy as np
import pytest

import oracle
from workloads import look_at, make_config, poses_sphere, scene_spheres
from workloads.configs import Camera

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
    """Every test of this module runs once per map layout."""
    c = nbt.Context(0)
    c.set_map_layout(request.param)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ig_close(ig, ref):
    ig = np.asarray(ig, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    both_nan = np.isnan(ig) & np.isnan(ref)
    rel = np.abs(ig - ref) / np.maximum(np.abs(ref), 1e-30)
    rel[both_nan] = 0.0
    zero = (ref == 0) & (ig == 0)
    rel[zero] = 0.0
    return float(np.nanmax(rel)) if rel.size else 0.0, bool(np.all(np.isnan(ig) == np.isnan(ref)))


def _compare_digests(d, ref):
    for key in ("steps", "stop_lin", "reason"):
        got = d[key].cpu().numpy().astype(np.int64)
        exp = ref[key].astype(np.int64)
        bad = np.argwhere(got != exp)
        assert bad.size == 0, f"{key} differs at {bad[:5].tolist()}: got {got[tuple(bad[0])]} want {exp[tuple(bad[0])]}"
    h = d["hash"].cpu().numpy().view(np.uint64)
    assert np.array_equal(h, ref["hash"]), f"hash differs at {np.argwhere(h != ref['hash'])[:5].tolist()}"
    g = d["gain"].cpu().numpy()
    ok = (g == ref["gain"]) | (np.isnan(g) & np.isnan(ref["gain"]))
    assert ok.all(), f"ray gain differs at {np.argwhere(~ok)[:5].tolist()}"


def _map(nbt, ctx, scene, thresholds=(0.5, 0.5)):
    return nbt.Map(ctx, scene.P, scene.voxel, scene.origin, thresholds=thresholds)


def test_cfg1_ray_digests_bit_exact(nbt, ctx):
    import torch
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note(f"cfg1 digests: {poses.shape[0]} poses x {cam.rays} rays")
    m = _map(nbt, ctx, scene)
    d = nbt.trace_rays(m, cam, _dev(poses))
    torch.cuda.synchronize()
    ref = oracle.trace_rays(scene, cam, poses)
    _compare_digests(d, ref)
    assert np.count_nonzero(ref["reason"] == oracle.RAY_HIT) > 100


def test_cfg1_ig_and_steps(nbt, ctx):
    import torch
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note("cfg1 eval_viewpoints")
    m = _map(nbt, ctx, scene)
    ig, st = nbt.eval_viewpoints(m, cam, _dev(poses))
    torch.cuda.synchronize()
    ig_ref, st_ref = oracle.eval_viewpoints(scene, cam, poses)
    assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref)
    rel, nan_ok = _ig_close(ig.cpu().numpy(), ig_ref)
    assert nan_ok and rel <= IG_RTOL, rel


@pytest.mark.parametrize("shape", [(1, 3, 1, 0, 1), (2, 3, 2, 1, 2), (4, 4, 1, 1, 4), (8, 2, 3, 0, 8),
                                   (4, 6, 1, 1, 1), (4, 0, 2, 1, 4), (8, 3, 8, 1, 2), (1, 3, 5, 1, 8),
                                   (8, 3, 0, 0, 4), (2, 5, 0, 1, 2)])
def test_launch_shapes_agree(nbt, ctx, shape):
    import torch
    waves, twl, tpw, remap, depth = shape
    sc = scene_spheres(n=(48, 40, 36), voxel=0.06, n_spheres=18, seed=301, origin=(-1.0, 0.5, 0.25))
    cam = Camera(37, 23, 64, 48, 1.7)           # ragged: not a multiple of any tile side
    poses = poses_sphere(sc.poi, 0.7, 21, seed=302)
    _note(f"launch shape {shape}")
    m = _map(nbt, ctx, sc)
    ctx.set_launch(waves, twl, tpw, remap, depth)
    try:
        ig, st = nbt.eval_viewpoints(m, cam, _dev(poses))
        torch.cuda.synchronize()
    finally:
        ctx.set_launch()
    ig_ref, st_ref = oracle.eval_viewpoints(sc, cam, poses)
    assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref)
    rel, nan_ok = _ig_close(ig.cpu().numpy(), ig_ref)
    assert nan_ok and rel <= IG_RTOL
    # without steps_out the kernel does not count visits; the IG is the same bits
    ctx.set_launch(waves, twl, tpw, remap, depth)
    try:
        ig2, _ = nbt.eval_viewpoints(m, cam, _dev(poses), want_steps=False)
        torch.cuda.synchronize()
    finally:
        ctx.set_launch()
    assert np.array_equal(ig2.cpu().numpy().view(np.uint32), ig.cpu().numpy().view(np.uint32))


def test_edge_cases(nbt, ctx):
    import torch
    _note("edge cases")
    n = 20
    P = np.full((n, n, n), 0.5, dtype=np.float32)
    P[5:8, 5:8, 5:8] = 1.0          # occupied with zero gain
    P[10:14, 2:6, 3:9] = 0.0        # free with zero gain
    P[0, :, :] = 0.9
    P[:, :, 15] = 0.2

    class S:
        pass
    sc = S()
    sc.P, sc.voxel, sc.origin = P, 0.1, np.array([0.3, -0.2, 0.1], np.float32)
    centre = sc.origin.astype(np.float64) + 1.0
    cams = [Camera(1, 1, 40, 30, 1.5), Camera(1, 9, 40, 30, 1.5), Camera(13, 1, 50, 30, 3.0),
            Camera(29, 17, 90, 70, 0.4)]
    pos = np.array([
        centre,                                   # inside the map
        centre + [0.0, 0.0, 5.0],                 # far outside, looking at the map
        sc.origin + [0.65, 0.65, 0.65],           # inside the occupied block
        sc.origin + [-0.5, -0.5, -0.5],           # outside a corner
    ])
    poses = look_at(pos, centre)
    away = look_at(centre[None] + [[0.0, 0.0, 5.0]], centre[None] + [[0.0, 0.0, 10.0]])
    nanpose = poses[:1].copy()
    nanpose[0, 4] = np.nan
    allp = np.concatenate([poses, away, nanpose], axis=0)
    for thr in [(0.5, 0.5), (0.7, 0.3)]:
        m = _map(nbt, ctx, sc, thresholds=thr)
        for cam in cams:
            ig, st = nbt.eval_viewpoints(m, cam, _dev(allp))
            d = nbt.trace_rays(m, cam, _dev(allp))
            torch.cuda.synchronize()
            ig_ref, st_ref = oracle.eval_viewpoints(sc, cam, allp, thresholds=thr)
            assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref)
            rel, nan_ok = _ig_close(ig.cpu().numpy(), ig_ref)
            assert nan_ok and rel <= IG_RTOL, (thr, cam)
            _compare_digests(d, oracle.trace_rays(sc, cam, allp, thresholds=thr))
            assert ig.cpu().numpy()[4] == 0.0 and math.isnan(ig.cpu().numpy()[5])
    # empty call is a no-op
    out = torch.full((1,), 7.0, device="cuda")
    nbt.binding._check(nbt.binding.lib().nbt_ig_eval_viewpoints(m.handle, nbt.camera(cams[0]),
                                                                 None, 0, None, None, None))
    assert out.item() == 7.0


def test_tiny_and_flat_maps(nbt, ctx):
    import torch
    _note("tiny maps")
    rng = np.random.default_rng(5)
    for dims in [(1, 1, 1), (7, 1, 1), (1, 5, 9), (3, 4, 2)]:
        nx, ny, nz = dims
        P = rng.choice(np.array([0.1, 0.5, 0.95], np.float32), size=(nz, ny, nx))

        class S:
            pass
        sc = S()
        sc.P, sc.voxel, sc.origin = P, 0.5, np.zeros(3, np.float32)
        c = np.array([nx, ny, nz]) * 0.25
        pos = c + rng.normal(size=(9, 3)) * 1.5
        poses = look_at(pos, c + rng.normal(size=3) * 0.2)
        cam = Camera(11, 7, 80, 60, 4.0)
        m = _map(nbt, ctx, sc)
        ig, st = nbt.eval_viewpoints(m, cam, _dev(poses))
        d = nbt.trace_rays(m, cam, _dev(poses))
        torch.cuda.synchronize()
        ig_ref, st_ref = oracle.eval_viewpoints(sc, cam, poses)
        assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref), dims
        rel, nan_ok = _ig_close(ig.cpu().numpy(), ig_ref)
        assert nan_ok and rel <= IG_RTOL
        _compare_digests(d, oracle.trace_rays(sc, cam, poses))


def test_cfg2_full_size_sampled(nbt, ctx):
    """Config 2 at its real size in the default launch shape: all 4096 perspectives
    on the GPU, the oracle on a seeded sample of them and of single rays."""
    import torch
    w = make_config(2)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note(f"cfg2 full size: {poses.shape[0]} poses, map {scene.P.shape}")
    m = _map(nbt, ctx, scene)
    dposes = _dev(poses)
    ig, st = nbt.eval_viewpoints(m, cam, dposes)
    ig2, st2 = nbt.eval_viewpoints(m, cam, dposes)
    torch.cuda.synchronize()
    ig, st = ig.cpu().numpy(), st.cpu().numpy().view(np.uint64)
    assert np.array_equal(ig, ig2.cpu().numpy()) and np.array_equal(st, st2.cpu().numpy().view(np.uint64))
    rng = np.random.default_rng(2025)
    pick = np.sort(rng.choice(poses.shape[0], size=6, replace=False))
    ig_ref, st_ref = oracle.eval_viewpoints(scene, cam, poses[pick])
    assert np.array_equal(st[pick], st_ref)
    rel, nan_ok = _ig_close(ig[pick], ig_ref)
    assert nan_ok and rel <= IG_RTOL
    # single rays: full voxel sequences
    sel = np.stack([rng.integers(0, poses.shape[0], 300), rng.integers(0, cam.rays, 300)], axis=1)
    lin, ln = nbt.trace_paths(m, cam, dposes, torch.from_numpy(sel.astype(np.int32)), 600)
    torch.cuda.synchronize()
    lin, ln = lin.cpu().numpy(), ln.cpu().numpy()
    for r, (p, k) in enumerate(sel):
        ref = oracle.cast_ray(scene, cam, poses[p], int(k) % cam.width, int(k) // cam.width)
        assert ln[r] == ref["steps"]
        assert np.array_equal(lin[r, :ln[r]], ref["path"])


def test_permutation_and_duplicates(nbt, ctx):
    import torch
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    m = _map(nbt, ctx, scene)
    perm = np.random.default_rng(9).permutation(poses.shape[0])
    both = np.concatenate([poses, poses[perm]], axis=0)
    ig, st = nbt.eval_viewpoints(m, cam, _dev(both))
    torch.cuda.synchronize()
    ig, st = ig.cpu().numpy(), st.cpu().numpy()
    n = poses.shape[0]
    assert np.array_equal(ig[n:], ig[:n][perm]) and np.array_equal(st[n:], st[:n][perm])


def test_argument_errors(nbt, ctx):
    import torch
    _note("argument errors")
    P = np.full((4, 4, 4), 0.5, np.float32)
    P[1, 2, 3] = np.nan
    with pytest.raises(nbt.NbtError) as e:
        nbt.Map(ctx, P, 0.1, (0, 0, 0))
    assert e.value.status == nbt.binding.EINVAL
    P[1, 2, 3] = 1.5
    with pytest.raises(nbt.NbtError):
        nbt.Map(ctx, P, 0.1, (0, 0, 0))
    P[1, 2, 3] = 0.5
    with pytest.raises(nbt.NbtError):
        nbt.Map(ctx, P, 0.1, (0, 0, 0), thresholds=(0.3, 0.7))
    with pytest.raises(nbt.NbtError):
        nbt.Map(ctx, P, -0.1, (0, 0, 0))
    m = nbt.Map(ctx, P, 0.1, (0, 0, 0))
    poses = _dev(look_at(np.array([[0.2, 0.2, 0.9]]), np.array([0.2, 0.2, 0.2])))
    for bad in [(0, 4, 0.5, 0.5, 1.0), (4, 4, 0.0, 0.5, 1.0), (4, 4, 0.5, 0.5, float("inf"))]:
        with pytest.raises(nbt.NbtError) as e:
            nbt.eval_viewpoints(m, bad, poses)
        assert e.value.status == nbt.binding.EINVAL
    with pytest.raises(nbt.NbtError):
        ctx.set_launch(3, 3, 1, 1)
    with pytest.raises(nbt.NbtError):
        ctx.set_launch(4, 3, -1, 0, 4)
    ig, _ = nbt.eval_viewpoints(m, (4, 4, 0.5, 0.5, 1.0), poses)
    torch.cuda.synchronize()
    assert np.isfinite(ig.cpu().numpy()).all()


def test_layouts_bit_identical(nbt, ctx):
    """Every storage order gives the same bits for IG, step counts and ray digests."""
    import torch
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note("layouts agree")
    out = {}
    before = ctx.get_map_layout()
    try:
        for lay in (0, 1, 2, 3):
            ctx.set_map_layout(lay)
            m = _map(nbt, ctx, scene)
            assert m.info()["layout"] == lay
            ig, st = nbt.eval_viewpoints(m, cam, _dev(poses))
            d = nbt.trace_rays(m, cam, _dev(poses))
            torch.cuda.synchronize()
            out[lay] = (ig.cpu().numpy().view(np.uint32), st.cpu().numpy(), d["hash"].cpu().numpy(),
                        d["steps"].cpu().numpy())
            m.close()
    finally:
        ctx.set_map_layout(before)
    for lay in (1, 2, 3):
        for a, b in zip(out[0], out[lay]):
            assert np.array_equal(a, b), lay
    with pytest.raises(nbt.NbtError):
        ctx.set_map_layout(4)


def test_relayout_and_layout_autotune(nbt, ctx):
    """Rewriting a map in another order keeps every result bit; the layout autotuner leaves
    the map in one of the two orders with the same results; a batch pins the order."""
    import torch
    w = make_config(1)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _note("relayout")
    m = _map(nbt, ctx, scene)
    dp = _dev(poses)
    ig0, st0 = nbt.eval_viewpoints(m, cam, dp)
    d0 = nbt.trace_rays(m, cam, dp)
    torch.cuda.synchronize()
    start = m.info()["layout"]
    for lay in ((start + 1) % 4, (start + 2) % 4, (start + 3) % 4, start):
        m.set_layout(lay)
        assert m.info()["layout"] == lay
        ig, st = nbt.eval_viewpoints(m, cam, dp)
        d = nbt.trace_rays(m, cam, dp)
        torch.cuda.synchronize()
        assert np.array_equal(ig.cpu().numpy().view(np.uint32), ig0.cpu().numpy().view(np.uint32))
        assert np.array_equal(st.cpu().numpy(), st0.cpu().numpy())
        assert np.array_equal(d["hash"].cpu().numpy(), d0["hash"].cpu().numpy())
    before = ctx.get_launch()
    try:
        launch, lay, ms = nbt.autotune_map(m, cam, dp)
        assert lay in (0, 1, 2, 3) and m.info()["layout"] == lay and ms > 0
        ig, st = nbt.eval_viewpoints(m, cam, dp)
        torch.cuda.synchronize()
        assert np.array_equal(ig.cpu().numpy().view(np.uint32), ig0.cpu().numpy().view(np.uint32))
    finally:
        ctx.set_launch(*[before[k] for k in ("waves_per_group", "tile_w_log2", "tiles_per_wave",
                                             "xcd_remap", "pipeline_depth")])
    b = nbt.Batch(ctx, [m], cam, 64)
    with pytest.raises(nbt.NbtError):
        m.set_layout((m.info()["layout"] + 1) % 4)
    b.close()
    m.set_layout((m.info()["layout"] + 1) % 4)  # allowed again once the batch is gone
    m.close()


def test_update_map_and_check(nbt, ctx):
    """Re-encoding a resident map in place from new probabilities gives the oracle's results on
    the new map; an update that meets NaN or values outside [0, 1] is reported by the next
    check (and only then), and a clean update afterwards checks clean."""
    import torch
    _note("map update + check")
    a = scene_spheres(n=(40, 36, 44), voxel=0.05, n_spheres=12, seed=311)
    b = scene_spheres(n=(40, 36, 44), voxel=0.05, n_spheres=25, seed=312)
    cam = Camera(37, 23, 60, 45, 1.5)
    poses = poses_sphere(a.poi, 0.6, 12, seed=313)
    m = nbt.Map(ctx, a.P, a.voxel, a.origin)
    dp = _dev(poses)
    m.update(_dev(b.P))
    ig, st = nbt.eval_viewpoints(m, cam, dp)
    torch.cuda.synchronize()
    m.check()
    ig_ref, st_ref = oracle.eval_viewpoints(b, cam, poses)
    assert np.array_equal(st.cpu().numpy().view(np.uint64), st_ref)
    rel, nan_ok = _ig_close(ig.cpu().numpy(), ig_ref)
    assert nan_ok and rel <= IG_RTOL
    bad = b.P.copy()
    bad[3, 4, 5] = np.nan
    bad[7, 8, 9] = 1.5
    m.update(_dev(bad))
    with pytest.raises(nbt.NbtError) as e:
        m.check()
    assert e.value.status == nbt.binding.EINVAL
    m.update(_dev(a.P))
    m.check()                                   # the flag was cleared by the failing check
    ig2, st2 = nbt.eval_viewpoints(m, cam, dp)
    torch.cuda.synchronize()
    ig_a, st_a = oracle.eval_viewpoints(a, cam, poses)
    assert np.array_equal(st2.cpu().numpy().view(np.uint64), st_a)
    with pytest.raises(ValueError):
        m.update(_dev(a.P[:-1]))
    m.close()
