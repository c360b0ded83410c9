"""The planner-facing calls under HIP graph capture: per-perspective IG, trajectory union IG,
the surrogate's selection and top-k, each captured once (after an eager call that sizes the
library's buffers) and replayed three times with eager work and synchronisations between the
replays.  Bar: every replay's outputs equal the eager call's bit for bit (outputs are
overwritten with -1 before each replay, so a replay that writes nothing fails).  None of
these calls reads anything back to the host or records a memset node.
"""

import sys

import numpy as np
import pytest

from workloads import make_config, poses_shell, trajectories_walk

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_22588_amd as nbt
    ctx = nbt.Context(0)
    w = make_config(1)
    sc = w.maps[0]
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    yield nbt, ctx, w, sc, m
    m.close()
    ctx.close()


def _replay_and_check(capture, eager_outs):
    """Capture `capture` (returns its output tensors) into a graph, replay it three times and
    compare each replay with the eager outputs, bit for bit."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        outs = capture()
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager_outs):
            assert torch.equal(o.view(torch.int8), e.view(torch.int8)), rep
        _ = torch.ones(4096, device="cuda").sum().item()      # eager work between replays
    del g


def test_viewpoints_in_a_graph(env):
    import torch
    nbt, ctx, w, sc, m = env
    _note("graph: eval_viewpoints, 64^3 map, 512 perspectives")
    poi = np.asarray(sc.poi, np.float64)
    dp = torch.from_numpy(poses_shell(poi, 0.4, 1.3, 512, 430)).cuda()
    ig, st = nbt.eval_viewpoints(m, w.camera, dp)
    torch.cuda.synchronize()
    _replay_and_check(lambda: nbt.eval_viewpoints(m, w.camera, dp), (ig.clone(), st.clone()))


def test_trajectories_in_a_graph(env):
    import torch
    nbt, ctx, w, sc, m = env
    _note("graph: eval_trajectories, 64^3 map, 24 trajectories x 6 poses")
    traj = trajectories_walk(sc.poi, 24, 6, seed=431)
    dt = torch.from_numpy(traj).cuda()
    ig, counts, visits = nbt.eval_trajectories(m, w.camera, dt)
    torch.cuda.synchronize()
    _replay_and_check(lambda: nbt.eval_trajectories(m, w.camera, dt), (ig.clone(), counts.clone(), visits.clone()))


def test_surrogate_select_and_top_k_in_a_graph(env):
    import os
    import torch
    nbt, ctx, w, sc, m = env
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2503_22588_amd", "weights", "surrogate_cfg1.nbts")
    _note("graph: surrogate select (8192 candidates, k_rescore 64) and top_k")
    sur = nbt.Surrogate(ctx, open(path, "rb").read())
    try:
        poi = np.asarray(sc.poi, np.float32)
        dp = torch.from_numpy(poses_shell(poi.astype(np.float64), 0.4, 1.3, 8192, 432)).cuda()
        idx, sig = sur.select(m, w.camera, poi, dp, k_rescore=64, k=10)
        torch.cuda.synchronize()
        _replay_and_check(lambda: sur.select(m, w.camera, poi, dp, k_rescore=64, k=10), (idx.clone(), sig.clone()))
        vals = torch.from_numpy(np.random.default_rng(433).standard_normal(20000).astype(np.float32)).cuda()
        ti, tv = nbt.top_k(ctx, vals, 37)
        torch.cuda.synchronize()
        _replay_and_check(lambda: nbt.top_k(ctx, vals, 37), (ti.clone(), tv.clone()))
    finally:
        sur.close()
