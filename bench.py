#!/usr/bin/env python
"""Throughput of per-perspective information gain on one MI355X.

Workload (the "plain raycast at scale" configuration): a 256^3 occupancy map
with 2 cm voxels of seeded table-top clutter (200 boxes and cylinders; the
unknown region is what three seeded prior cameras could not see), 4 points of
interest x 1024 perspectives sampled uniformly in the 0.5-1.2 m shell around
each, a 160x120 endpoint grid, 70x55 degree field of view and 3 m range.

One step = one information-distribution update: re-encode the resident map
from its probabilities (nbt_ig_update_map) and evaluate the IG of all 4096
perspectives (nbt_ig_eval_viewpoints).  Inputs are resident in HBM before the
timed region starts.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "viewpoint IG evals/s + voxel-steps/s vs L2/HBM roofline; surrogate vs raycast"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_STEP = 4             # one encoded map word gathered per visited voxel
BYTES_PER_VIEWPOINT = 48 + 4 + 8   # pose in, IG and step count out


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(scene, cam, poses, budget_s):
    """The oracle, single-threaded, on a seeded sample of the same perspectives."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(7)
    order = rng.permutation(poses.shape[0])
    t0 = time.perf_counter()
    oracle.eval_viewpoints(scene, cam, poses[order[:1]])
    one = max(time.perf_counter() - t0, 1e-3)
    k = int(min(max(2, budget_s / one), poses.shape[0]))
    sample = poses[order[:k]]
    t0 = time.perf_counter()
    _, steps = oracle.eval_viewpoints(scene, cam, sample)
    dt = time.perf_counter() - t0
    return {
        "value": k / dt,
        "unit": "viewpoint evals/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{k} of {poses.shape[0]} perspectives (seeded permutation), all "
                  f"{cam.width}x{cam.height} rays each; {int(steps.sum())} voxel steps in {dt:.1f} s "
                  f"on {platform.processor() or platform.machine()}",
        "voxel_steps_per_s": float(steps.sum()) / dt,
    }


def _timed(fn, reps, stream):
    """Mean milliseconds of fn() over reps launches (HIP events on `stream`)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def extra_trajectories(nbt, ctx, reps):
    """Trajectory IG: 256^3 sphere map, 4096 trajectories x 24 poses, 128x96 rays."""
    import numpy as np
    import torch
    from workloads import make_config
    w = make_config(4)
    sc, cam, traj = w.maps[0], w.camera, w.poses[0]
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    dt = torch.from_numpy(traj).cuda()
    out = {}

    def run():
        out["r"] = nbt.eval_trajectories(m, cam, dt)

    ms = _timed(run, reps, torch.cuda.current_stream())
    ig, counts, visits = out["r"]
    vis = int(visits.cpu().numpy().view(np.uint64).sum())
    rays = traj.shape[0] * traj.shape[1] * cam.width * cam.height
    return {"workload": "256^3 map (5 cm, 1280 spheres), 4096 trajectories x 24 poses, 128x96 rays",
            "ms_per_launch": ms, "trajectory_evals_per_s": traj.shape[0] / (ms * 1e-3),
            "rays_per_s": rays / (ms * 1e-3), "voxel_steps_per_s": vis / (ms * 1e-3),
            "mean_unique_voxels": float(counts[:, 0].float().mean().item()),
            "note": "includes the box pre-pass and its one host synchronisation"}


def extra_batch(nbt, ctx, reps):
    """Batched: 64 maps of {64..256}^3, log-uniform 16-2048 perspectives each, one graph launch."""
    import numpy as np
    import torch
    from workloads import make_config
    w = make_config(3)
    maps = [nbt.Map(ctx, s.P, s.voxel, s.origin) for s in w.maps]
    counts = [p.shape[0] for p in w.poses]
    offsets = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)).cuda()
    allp = torch.from_numpy(np.concatenate(w.poses, axis=0)).cuda()
    n = allp.shape[0]
    ig = torch.empty(n, device="cuda")
    st = torch.empty(n, dtype=torch.int64, device="cuda")
    b = nbt.Batch(ctx, maps, w.camera, n)
    best, _ = b.autotune(offsets, allp, ig, st)
    ms = _timed(lambda: b.run(offsets, allp, ig, st), reps, torch.cuda.current_stream())
    steps = int(st.cpu().numpy().view(np.uint64).sum())
    rays = n * w.camera.width * w.camera.height
    res = {"workload": f"64 maps (sizes in {{64,96,128,192,256}}^3, 5 cm), {n} perspectives, 64x48 rays",
           "batch_latency_ms": ms, "viewpoint_evals_per_s": n / (ms * 1e-3), "rays_per_s": rays / (ms * 1e-3),
           "voxel_steps_per_s": steps / (ms * 1e-3), "launch": b.get_launch()}
    b.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="waves,tile_w_log2,tiles_per_wave,xcd_remap,pipeline_depth")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the trajectory and batched measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE={world}) is not supported: "
              "the IG evaluation shards by perspective with no exchange, and this build runs on a "
              "single MI355X.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "dispatches": 5}), flush=True)
        return

    import paper_2503_22588_amd as nbt
    from workloads import make_config

    t_gen = time.perf_counter()
    w = make_config(2)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _log(f"workload generated in {time.perf_counter() - t_gen:.1f} s: map {scene.P.shape}, "
         f"{poses.shape[0]} perspectives, {cam.width}x{cam.height} rays")

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = nbt.Context(0)
    if args.launch:
        ctx.set_launch(*[int(v) for v in args.launch.split(",")])
    prob = torch.from_numpy(scene.P).cuda()
    m = nbt.Map(ctx, prob, scene.voxel, scene.origin)
    dposes = torch.from_numpy(poses).cuda()
    n = poses.shape[0]
    ig = torch.empty(n, dtype=torch.float32, device="cuda")
    steps = torch.empty(n, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def step():
        m.update(prob)
        nbt.eval_viewpoints(m, cam, dposes, ig_out=ig, steps_out=steps)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    m.check()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        m.update(prob)
        e1.record(stream)
        nbt.eval_viewpoints(m, cam, dposes, ig_out=ig, steps_out=steps)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    enc_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    ray_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    total_steps = int(steps.cpu().numpy().view(np.uint64).sum())
    ms_per_step = wall * 1e3 / args.steps
    evals_per_s = n * args.steps / wall
    rays = n * cam.width * cam.height

    alg_bytes = BYTES_PER_STEP * total_steps + BYTES_PER_VIEWPOINT * n
    achieved_gbs = alg_bytes / (ray_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": evals_per_s,
        "unit": "viewpoint evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "plain raycast at scale: 256^3 table-top map (2 cm voxels, 200 objects, "
                        "unknown = hidden from 3 prior views), 4 PoIs x 1024 perspectives in the "
                        "0.5-1.2 m shell, 160x120 rays, 70x55 deg, 3 m range",
            "perspectives": n,
            "rays_per_perspective": cam.width * cam.height,
            "map": list(scene.P.shape[::-1]),
            "launch": ctx.get_launch(),
        },
        "rays_per_s": rays * args.steps / wall,
        "voxel_steps_per_s": total_steps * args.steps / wall,
        "voxel_steps_per_step": total_steps,
        "kernel_ms": {"encode_map": enc_ms, "ig_viewpoints": ray_ms},
        "roofline": {
            "kernel": "ig_viewpoints_kernel",
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": None,
        },
    }
    if not args.no_extras:
        _log("measuring trajectory IG (config 4) ...")
        result["trajectories"] = extra_trajectories(nbt, ctx, reps=3)
        _log("measuring the batched launch (config 3) ...")
        result["batched"] = extra_batch(nbt, ctx, reps=5)
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(scene, cam, poses, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
