"""The no-allocation per-perspective entry point (nbt_ig_eval_viewpoints_noalloc) against the
allocating one (nbt_ig_eval_viewpoints), through the C ABI.

Both run the same kernels; only where the cross-workgroup reduction slots live differs (a
fixed array the library holds per device instead of the context's workspace), so IG and step
counts must agree bit for bit, call after call, including a second, smaller call that finds
the first call's slots in the array.  A sample is also checked against the oracle (steps
exact, IG within 1e-5 relative).
"""

import numpy as np
import pytest

import oracle
from workloads import poses_sphere, scene_spheres
from workloads.configs import Camera

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


@pytest.fixture(scope="module")
def setup(nbt):
    ctx = nbt.Context(0)
    sc = scene_spheres(n=(96, 80, 88), voxel=0.04, n_spheres=40, seed=7401)
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    yield ctx, sc, m
    m.close()
    ctx.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(nbt, m, cam, poses, want_steps=True):
    import torch
    n = poses.shape[0]
    ig_a, st_a = nbt.eval_viewpoints(m, cam, poses, want_steps=want_steps)
    ig_b = torch.full((n,), -7.0, dtype=torch.float32, device=poses.device)
    st_b = torch.full((n,), -7, dtype=torch.int64, device=poses.device) if want_steps else None
    nbt.eval_viewpoints_noalloc(m, cam, poses, ig_b, st_b)
    torch.cuda.synchronize()
    assert np.array_equal(ig_a.cpu().numpy().view(np.int32), ig_b.cpu().numpy().view(np.int32))
    if want_steps:
        assert np.array_equal(st_a.cpu().numpy(), st_b.cpu().numpy())
    return ig_b.cpu().numpy(), (st_b.cpu().numpy() if want_steps else None)


@pytest.mark.parametrize("cam", [Camera(160, 120, 70.0, 55.0, 3.0), Camera(64, 48, 60.0, 45.0, 2.0)],
                         ids=["160x120", "64x48"])
def test_two_calls_second_smaller(nbt, setup, cam):
    ctx, sc, m = setup
    _note(f"noalloc: {cam.width}x{cam.height}, 300 then 37 perspectives")
    poses = poses_sphere(sc.poi, 1.1, 300, seed=7402)
    dp = _dev(poses)
    ig1, st1 = _pair(nbt, m, cam, dp)
    ig2, st2 = _pair(nbt, m, cam, dp[100:137])
    assert np.array_equal(ig2.view(np.int32), ig1[100:137].view(np.int32))
    assert np.array_equal(st2, st1[100:137])
    _pair(nbt, m, cam, dp[:5], want_steps=False)
    # the oracle on a sample of the first call
    sample = np.array([0, 57, 199, 299])
    ig_ref, st_ref = oracle.eval_viewpoints(sc, cam, poses[sample])
    assert np.array_equal(st1[sample].astype(np.uint64), st_ref)
    rel = np.abs(ig1[sample].astype(np.float64) - ig_ref) / np.maximum(np.abs(ig_ref), 1e-30)
    assert rel.max() <= 1e-5


def test_limit_and_errors(nbt, setup):
    import torch
    ctx, sc, m = setup
    cam = Camera(16, 12, 60.0, 45.0, 2.0)
    n = nbt.binding.NOALLOC_MAX_VIEWPOINTS + 1
    poses = torch.zeros((n, 12), dtype=torch.float32, device="cuda")
    ig = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(nbt.NbtError) as e:
        nbt.eval_viewpoints_noalloc(m, cam, poses, ig)
    assert e.value.status == nbt.binding.EUNSUPPORTED
    torch.cuda.synchronize()
    assert not ig.any()                                      # nothing was launched
    # at the limit, every slot in use: 72x64 rays are 72 tiles of 8x8, two workgroups per perspective
    cam = Camera(72, 64, 60.0, 45.0, 1.0)
    _note("noalloc: 65536 perspectives")
    poses = _dev(poses_sphere(sc.poi, 1.0, n - 1, seed=7403))
    ig_full, st_full = _pair(nbt, m, cam, poses)
    assert np.isfinite(ig_full).all() and (st_full > 0).all()
    # n == 0 is a no-op
    nbt.eval_viewpoints_noalloc(m, cam, poses[:0], ig[:0])
