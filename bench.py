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


# Sources that decide the ray kernel's binary, its launch shape and the
# benchmark workload: counter results taken for one fingerprint are reported
# only while it still matches.
FINGERPRINT_FILES = (
    "paper_2503_22588_amd/build.py",
    "paper_2503_22588_amd/csrc/ray.hpp",
    "paper_2503_22588_amd/csrc/raycast_viewpoints.hip",
    "paper_2503_22588_amd/csrc/internal.hpp",
    "paper_2503_22588_amd/csrc/host.hpp",
    "paper_2503_22588_amd/csrc/nbt_ig.hip",
    "paper_2503_22588_amd/csrc/map_encode.hip",
    "workloads/configs.py",
    "workloads/scenes.py",
    "workloads/poses.py",
)
COUNTERS_PROFILE = "profiles/ig_viewpoints_cfg2_counters.md"


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_fingerprint():
    """sha256 (first 16 hex digits) over the fingerprint files, in order."""
    import hashlib
    h = hashlib.sha256()
    for rel in FINGERPRINT_FILES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()[:16]


def launch_key(layout, launch):
    """'<map order> w,t,p,x,d': the map order and launch shape a counters summary was taken for."""
    return f"{layout} " + ",".join(str(launch[k]) for k in
                                   ("waves_per_group", "tile_w_log2", "tiles_per_wave", "xcd_remap",
                                    "pipeline_depth"))


def measured_counters(shape=None):
    """`key: value` lines of the committed counters summary for one map order and launch
    shape: the block that starts at `- launch: <shape>` (the first block when `shape` is
    None), with the summary's fingerprint.  None when the summary was taken for other
    sources than the ones built now, or holds no block for `shape`."""
    path = os.path.join(ROOT, COUNTERS_PROFILE)
    if not os.path.exists(path):
        return None
    common, blocks, cur = {}, [], None
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            k, v = k.strip(), v.strip().strip("`")
            if k == "launch":
                cur = {}
                blocks.append(cur)
            (common if cur is None else cur)[k] = v
    if common.get("fingerprint") != kernel_fingerprint() or not blocks:
        return None
    for b in blocks:
        if shape is None or b["launch"] == shape:
            return {**common, **b}
    return None


def cpu_identity():
    """The host CPU as lscpu names it, and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model or platform.processor() or platform.machine(),
            "nproc": os.cpu_count(), "cores_allowed": len(os.sched_getaffinity(0))}


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
    ident = cpu_identity()
    return {
        "value": k / dt,
        "unit": "viewpoint evals/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{k} of {poses.shape[0]} perspectives (seeded permutation), all "
                  f"{cam.width}x{cam.height} rays each; {int(steps.sum())} voxel steps in {dt:.1f} s "
                  f"on one core of {ident['cpu_model']} ({ident['nproc']} logical CPUs)",
        "voxel_steps_per_s": float(steps.sum()) / dt,
        **ident,
    }


def _oracle_other_workloads(core, conn):
    """Child process (started before this program touches the GPU), pinned to one core: the
    oracle on the 64^3 sphere workload and the 64-map batch in full, and on 64 of the 4096
    trajectories of the trajectory workload."""
    try:
        os.sched_setaffinity(0, {core})
        import numpy as np
        import oracle
        from workloads import make_config
        out = {}
        w = make_config(1)
        t0 = time.perf_counter()
        _, st = oracle.eval_viewpoints(w.maps[0], w.camera, w.poses[0])
        dt = time.perf_counter() - t0
        out["plain_64"] = {"workload": "64^3 sphere map, 32 perspectives, 64x48 rays (all)", "seconds": dt,
                           "viewpoint_evals_per_s": w.poses[0].shape[0] / dt,
                           "voxel_steps_per_s": float(st.sum()) / dt}
        w = make_config(3)
        t0 = time.perf_counter()
        tot, nv = 0, 0
        for sc, ps in zip(w.maps, w.poses):
            _, st = oracle.eval_viewpoints(sc, w.camera, ps)
            tot += int(st.sum())
            nv += ps.shape[0]
        dt = time.perf_counter() - t0
        out["batched"] = {"workload": f"64 maps, {nv} perspectives, 64x48 rays (all)", "seconds": dt,
                          "viewpoint_evals_per_s": nv / dt, "voxel_steps_per_s": tot / dt}
        w = make_config(4)
        sub = w.poses[0][np.random.default_rng(11).permutation(w.poses[0].shape[0])[:64]]
        t0 = time.perf_counter()
        _, _, visits = oracle.eval_trajectories(w.maps[0], w.camera, sub)
        dt = time.perf_counter() - t0
        out["trajectories"] = {"workload": "64 of the 4096 trajectories (seeded), 24 poses x 128x96 rays each",
                               "seconds": dt, "trajectory_evals_per_s": 64 / dt,
                               "voxel_steps_per_s": float(np.sum(visits)) / dt,
                               "note": "a subset: the rate per trajectory, not the full 4096"}
        conn.send(out)
    except Exception as e:  # reported in the JSON line, never fatal
        conn.send({"error": f"{type(e).__name__}: {e}"})
    finally:
        conn.close()


def start_other_baselines():
    """Starts _oracle_other_workloads on the last allowed core; returns (process, pipe)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    parent, child = ctx.Pipe(duplex=False)
    core = max(os.sched_getaffinity(0))
    p = ctx.Process(target=_oracle_other_workloads, args=(core, child), daemon=True)
    p.start()
    child.close()
    return p, parent


def finish_other_baselines(handle, timeout_s=240.0):
    p, conn = handle
    res = conn.recv() if conn.poll(timeout_s) else {"error": f"not done within {timeout_s:.0f} s"}
    p.join(5)
    if p.is_alive():
        p.terminate()
    return res


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


CEILING_SIZES = ((1 << 20, "1MiB"), (64 << 20, "64MiB"), (1 << 30, "1GiB"))


def measure_ceilings(nbt, ctx, reps=10):
    """Useful-byte rates of the library's memory probes (nbt_ig_probe_memory) over working sets
    that fit each XCD's L2 (1 MiB), that only the Infinity Cache holds (64 MiB: above the 8 x
    4 MiB of L2, within its 256 MiB) and that only HBM holds (1 GiB).  Gathers are 4-byte words
    at pseudo-random positions, one per lane (`gather`) or one 16-byte piece per quad
    (`quad_gather`, the coalescing best case of a 2x2 ray quad)."""
    import torch
    buf = torch.randint(-2 ** 31, 2 ** 31 - 1, ((1 << 30) // 4,), dtype=torch.int32, device="cuda")
    sink = nbt.binding.probe_memory(ctx, nbt.binding.PROBE_STREAM, buf[:4], 1)
    stream = torch.cuda.current_stream()
    lanes = 256 * 8 * ctx.info()["cu_count"]
    loads = 1024
    out = {}
    for size, label in CEILING_SIZES:
        b = buf[: size // 4]
        passes = max(1, (512 << 20) // size)
        ms = _timed(lambda: nbt.binding.probe_memory(ctx, nbt.binding.PROBE_STREAM, b, passes, sink), reps, stream)
        row = {"stream_gbs": passes * size / (ms * 1e-3) / 1e9}
        for name, kind in (("gather", nbt.binding.PROBE_GATHER), ("quad_gather", nbt.binding.PROBE_QUAD_GATHER)):
            ms = _timed(lambda: nbt.binding.probe_memory(ctx, kind, b, loads, sink), reps, stream)
            row[f"{name}_words_per_s"] = lanes * loads / (ms * 1e-3)
            row[f"{name}_gbs"] = 4 * lanes * loads / (ms * 1e-3) / 1e9
        out[label] = row
    del buf
    torch.cuda.empty_cache()
    return out


def level_fractions(steps_per_s, map_bytes, ceilings):
    """The walk's voxel-step rate (one 4-byte word per step) against the probes' rates at the
    working set closest to the map's size."""
    if not ceilings:
        return None
    label = "1MiB" if map_bytes <= (4 << 20) else ("64MiB" if map_bytes <= (192 << 20) else "1GiB")
    c = ceilings[label]
    level = {"1MiB": "L2", "64MiB": "Infinity Cache (MALL)", "1GiB": "HBM"}[label]
    return {"map_bytes": map_bytes, "level": level, "ceiling_working_set": label,
            "frac_vs_stream": 4 * steps_per_s / (c["stream_gbs"] * 1e9),
            "frac_vs_quad_gather": steps_per_s / c["quad_gather_words_per_s"],
            "frac_vs_gather": steps_per_s / c["gather_words_per_s"]}


BF16_PEAK_TFLOPS = 2500.0           # MI355X dense BF16 MFMA, datasheet
MLP_FLOP_PER_POSE = 2 * (256 * 256 + 256 * 4 + 256)   # fc2 + the per-pose part of fc1 + fc3


def measure_mfma_ceiling(nbt, ctx, reps=5, iters=2048):
    """TFLOP/s of the library's MFMA probe (nbt_ig_probe_mfma): independent BF16 chains in
    registers, both instruction forms, 1 and 2 waves per SIMD (the MLP runs 2)."""
    import torch
    stream = torch.cuda.current_stream()
    out = {}
    for name, kind in (("16x16x32", nbt.binding.PROBE_MFMA_16X16X32_BF16),
                       ("32x32x16", nbt.binding.PROBE_MFMA_32X32X16_BF16)):
        for w in (1, 2):
            sink, flops = nbt.binding.probe_mfma(ctx, kind, w, iters)
            ms = _timed(lambda: nbt.binding.probe_mfma(ctx, kind, w, iters, sink), reps, stream)
            out[f"{name}_bf16_{w}wave_tflops"] = flops / (ms * 1e-3) / 1e12
    return out


def roofline_of(kernel, steps_per_s, map_bytes, ceilings):
    """The contract's roofline object for a walk kernel: algorithmic bytes (4 per voxel step)
    against the HBM peak, plus the fractions of the measured ceilings of the map's level."""
    ach = 4 * steps_per_s / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None,
            "levels": level_fractions(steps_per_s, map_bytes, ceilings)}


def extra_trajectories(nbt, ctx, reps, ceilings=None):
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
        out["r"] = nbt.eval_trajectories(m, cam, dt, want_visits=False)

    # the library's defaults first, so that the line states what the tuner buys
    untuned = {"map_layout": nbt.LAYOUT_NAMES[m.info()["layout"]],
               "ms_per_launch": _timed(run, reps, torch.cuda.current_stream())}
    layout, waves, _ = nbt.autotune_trajectories(m, cam, dt)
    ms = _timed(run, reps, torch.cuda.current_stream())
    ig, counts, _ = out["r"]
    # visits from one untimed counting call, whose IG and counts must be the same bits
    ig_c, counts_c, visits = nbt.eval_trajectories(m, cam, dt)
    torch.cuda.synchronize()
    if not (torch.equal(ig_c.view(torch.int32), ig.view(torch.int32)) and torch.equal(counts_c, counts)):
        raise RuntimeError("trajectory IG or counts differ between the counting and the plain walk")
    vis = int(visits.cpu().numpy().view(np.uint64).sum())
    rays = traj.shape[0] * traj.shape[1] * cam.width * cam.height
    return {"workload": "256^3 map (5 cm, 1280 spheres), 4096 trajectories x 24 poses, 128x96 rays",
            "ms_per_launch": ms, "trajectory_evals_per_s": traj.shape[0] / (ms * 1e-3),
            "rays_per_s": rays / (ms * 1e-3), "voxel_steps_per_s": vis / (ms * 1e-3),
            "mean_unique_voxels": float(counts[:, 0].float().mean().item()),
            "map_layout": nbt.LAYOUT_NAMES[layout], "waves_per_group": waves,
            "untuned": untuned, "tuner_speedup": untuned["ms_per_launch"] / ms,
            "note": "timed without the visit count (its voxel steps come from one untimed counting call); "
                    "includes the box pre-pass; nothing is read back to the host",
            "roofline": roofline_of("traj_union_kernel", vis / (ms * 1e-3), int(m.info()["device_bytes"]),
                                    ceilings)}


def extra_insert(nbt, ctx, reps):
    """Map update: 16 depth scans of 640x576 inserted into a 256^3 log-odds grid (2 cm)."""
    import numpy as np
    import torch
    from workloads import poses_sphere, scene_spheres
    from workloads.configs import Camera
    from workloads.depth import depth_images
    sc = scene_spheres(n=256, voxel=0.02, n_spheres=60, seed=921, r_range=(0.08, 0.4))
    cam = Camera(640, 576, 75.0, 65.0, 3.0)
    poses = poses_sphere(sc.poi, 1.2, 16, seed=922)
    depth = depth_images(sc, cam, poses, invalid_frac=0.02, seed=923)
    m = nbt.Map(ctx, np.full(sc.P.shape, 0.5, np.float32), sc.voxel, sc.origin)
    L = torch.zeros(sc.P.shape, dtype=torch.float32, device="cuda")
    P = torch.empty_like(L)
    dp, dd = torch.from_numpy(poses).cuda(), torch.from_numpy(depth).cuda()
    stream = torch.cuda.current_stream()
    ms_ins = _timed(lambda: nbt.insert_scans(m, cam, dp, dd, L), reps, stream)

    def full():
        nbt.insert_scans(m, cam, dp, dd, L, prob_out=P)
        m.update(P)

    ms_full = _timed(full, reps, stream)
    m.check()
    rays = poses.shape[0] * cam.width * cam.height
    measured = int(np.count_nonzero(depth > 0))
    returns = int(np.count_nonzero((depth > 0) & (depth < cam.range)))
    m.close()
    return {"workload": "256^3 log-odds grid (2 cm, 60 spheres), 16 scans of 640x576 z-depth "
                        "(75x65 deg, 3 m), 2 % dropped pixels",
            "insert_ms": ms_ins, "scans_per_s": poses.shape[0] / (ms_ins * 1e-3),
            "rays_per_s": rays / (ms_ins * 1e-3), "measured_pixels": measured, "returns": returns,
            "update_ms": ms_full,
            "note": "insert_ms: the 16 scans into the log-odds grid; update_ms adds the probabilities "
                    "and the re-encoding of the map"}


def extra_batch(nbt, ctx, reps, ceilings=None):
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
    # the library's defaults first, so that the line states what the tuner buys
    untuned = {"launch": b.get_launch(), "map_layout": nbt.LAYOUT_NAMES[maps[0].info()["layout"]],
               "batch_latency_ms": _timed(lambda: b.run(offsets, allp, ig, st), reps,
                                          torch.cuda.current_stream())}
    layout, _ = b.autotune_layout(offsets, allp, ig, st)     # untimed set-up: map order, then shape
    best, _ = b.autotune(offsets, allp, ig, st)
    ms = _timed(lambda: b.run(offsets, allp, ig, st), reps, torch.cuda.current_stream())
    steps = int(st.cpu().numpy().view(np.uint64).sum())
    rays = n * w.camera.width * w.camera.height
    res = {"workload": f"64 maps (sizes in {{64,96,128,192,256}}^3, 5 cm), {n} perspectives, 64x48 rays",
           "batch_latency_ms": ms, "viewpoint_evals_per_s": n / (ms * 1e-3), "rays_per_s": rays / (ms * 1e-3),
           "voxel_steps_per_s": steps / (ms * 1e-3), "launch": b.get_launch(),
           "map_layout": nbt.LAYOUT_NAMES[layout],
           "untuned": untuned, "tuner_speedup": untuned["batch_latency_ms"] / ms,
           "roofline": roofline_of("ig_batch_kernel", steps / (ms * 1e-3),
                                   sum(int(mm.info()["device_bytes"]) for mm in maps), ceilings)}
    b.close()
    return res


def extra_top_k(nbt, ctx, reps=20):
    """Next-best-view selection (nbt_ig_top_k): the k best of n per-perspective IG values, best
    first, ties to the lower index; n = 4096 (one call of the headline workload), 65,536 and
    2^20 seeded values with ties."""
    import numpy as np
    import torch
    rng = np.random.default_rng(17)
    stream = torch.cuda.current_stream()
    rows = []
    for n, ks in ((4096, (1, 10)), (65536, (10, 256)), (1 << 20, (10, 1024))):
        v = torch.from_numpy(np.round(rng.gamma(2.0, 0.1, n), 3).astype(np.float32)).cuda()
        for k in ks:
            ms = _timed(lambda: nbt.top_k(ctx, v, k), reps, stream)
            rows.append({"n": n, "k": k, "us_per_call": ms * 1e3, "values_per_s": n / (ms * 1e-3)})
    return {"workload": "k best of n IG values (gamma-distributed, rounded to 1e-3: many ties)", "rows": rows}


def _held_out_map(family, i):
    """(P, voxel, origin, poi, shell, camera, seed) of held-out map i of a surrogate family (seeds
    outside the training ranges of paper_2503_22588_amd/train_surrogate.py and outside the
    held-out sets that chose among training runs)."""
    import numpy as np
    from workloads import scene_spheres, scene_tabletop
    from workloads.configs import CAM1, CAM2
    if family == "cfg1":
        seed = 22588 + 5000 + 400000 + i
        sc = scene_spheres(n=64, voxel=0.05, n_spheres=10 + seed % 31, seed=seed)
        return sc.P, sc.voxel, sc.origin, np.asarray(sc.poi, np.float32), (0.4, 1.3), CAM1, seed
    seed = 22588 + 6000 + 400000 + i
    sc = scene_tabletop(n=256, voxel=0.02, n_objects=200, seed=seed)
    tops = sc.extra["object_tops"]
    poi = np.asarray(tops[np.random.default_rng(seed + 77).choice(len(tops), size=4, replace=False)[0]], np.float32)
    return sc.P, sc.voxel, sc.origin, poi, (0.5, 1.2), CAM2, seed


def extra_surrogate(nbt, ctx, family="cfg1", n_maps=32, n_cand=65536, k_rescores=(64, 256, 1024), k=10,
                    target=0.95):
    """Surrogate-pruned selection vs plain raycasting on held-out maps of one scene family
    (cfg1: 64^3 sphere maps, cfg2: 256^3 table-top maps), at several rescoring budgets; the
    headline operating point is the smallest budget whose top-10 agreement with exact IG
    reaches `target`."""
    import numpy as np
    import torch
    from workloads import poses_shell
    path = os.path.join(ROOT, "paper_2503_22588_amd", "weights", f"surrogate_{family}.nbts")
    if not os.path.exists(path):
        return {"skipped": f"no trained weights at {os.path.relpath(path, ROOT)}"}
    blob = open(path, "rb").read()
    sur = nbt.Surrogate(ctx, blob)
    stream = torch.cuda.current_stream()
    t_plain, nmae, t_mlp = [], [], []
    per = {kr: {"agree": [], "ratio": [], "ms": []} for kr in k_rescores}
    for i in range(n_maps):
        P, vox, origin, poi, shell, CAM, seed = _held_out_map(family, i)
        m = nbt.Map(ctx, P, vox, origin)
        if family == "cfg1":
            m.set_layout(nbt.LAYOUT_LINEAR)     # 5 cm map, dense rays: the linear order is faster
        dp = torch.from_numpy(poses_shell(poi.astype(np.float64), shell[0], shell[1], n_cand, seed + 500)).cuda()
        ig = torch.empty(n_cand, device="cuda")
        t_plain.append(_timed(lambda: nbt.eval_viewpoints(m, CAM, dp, ig_out=ig, want_steps=False), 3, stream))
        ex = ig.cpu().numpy()
        top = set(np.lexsort((np.arange(n_cand), -ex))[:k].tolist())
        sel_idx = torch.empty(k, dtype=torch.int32, device="cuda")
        sel_ig = torch.empty(k, device="cuda")
        for kr in k_rescores:
            out = {}

            def sel():
                out["r"] = sur.select(m, CAM, poi, dp, k_rescore=kr, k=k, idx_out=sel_idx, ig_out=sel_ig)

            per[kr]["ms"].append(_timed(sel, 5, stream))
            per[kr]["agree"].append(len(top & set(out["r"][0].cpu().numpy().tolist())) / k)
            per[kr]["ratio"].append(float(out["r"][1].cpu().numpy()[0]) / float(ex.max()))
        pred = sur.predict(m, poi, dp)
        # the MLP alone: prediction (trunk + MLP) minus the trunk (features with no outputs)
        if i < 4:
            t_mlp.append(_timed(lambda: sur.predict(m, poi, dp, pred=pred), 20, stream)
                         - _timed(lambda: sur.features(m, poi, want_patch=False, want_features=False), 20, stream))
        torch.cuda.synchronize()
        nmae.append(float(np.mean(np.abs(pred.cpu().numpy() - ex)) / np.mean(ex)))
        m.close()
    sur.close()
    tp = float(np.mean(t_plain))
    points = []
    for kr in k_rescores:
        ts = float(np.mean(per[kr]["ms"]))
        points.append({"k_rescore": kr, "surrogate_ms": ts, "surrogate_evals_per_s": n_cand / (ts * 1e-3),
                       "speedup": tp / ts, "top10_agreement": float(np.mean(per[kr]["agree"])),
                       "best_ig_ratio": float(np.mean(per[kr]["ratio"])),
                       "worst_best_ig_ratio": float(np.min(per[kr]["ratio"]))})
    ok = [p for p in points if p["top10_agreement"] >= target]
    head = ok[0] if ok else points[-1]
    desc = {"cfg1": f"{n_maps} held-out 64^3 sphere maps (5 cm), {n_cand} candidates in the 0.4-1.3 m shell, "
                    f"64x48 rays",
            "cfg2": f"{n_maps} held-out 256^3 table-top maps (2 cm, f = 5 crop), {n_cand} candidates in the "
                    f"0.5-1.2 m shell around an object top, 160x120 rays"}[family]
    return {"workload": f"{desc}; top-k_rescore rescored exactly, top-{k} kept",
            "plain_ms": tp, "plain_evals_per_s": n_cand / (tp * 1e-3),
            "k_rescore": head["k_rescore"], "surrogate_ms": head["surrogate_ms"],
            "surrogate_evals_per_s": head["surrogate_evals_per_s"], "speedup": head["speedup"],
            "top10_agreement": head["top10_agreement"], "best_ig_ratio": head["best_ig_ratio"],
            "agreement_target": target, "operating_points": points,
            "prediction_nmae": float(np.mean(nmae)),
            "roofline": mlp_roofline(nbt, ctx, n_cand, float(np.mean(t_mlp)))}


def mlp_roofline(nbt, ctx, n_cand, mlp_ms):
    """The MLP's algorithmic FLOPs over its time, against the BF16 datasheet peak and against the
    MFMA probe's rate for the MLP's instruction form and occupancy (32x32x16, 2 waves per SIMD)."""
    ceil = measure_mfma_ceiling(nbt, ctx)
    if not mlp_ms > 0.0:              # a difference of two timings: noise must not make a rate of it
        return {"kernel": "mlp_kernel", "bound": "mfma", "achieved": None, "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": None, "traffic": None, "measured_mfma_tflops": ceil,
                "note": f"prediction minus trunk time was {mlp_ms} ms: not a usable MLP time"}
    ach = n_cand * MLP_FLOP_PER_POSE / (mlp_ms * 1e-3) / 1e12
    meas = ceil["32x32x16_bf16_2wave_tflops"]
    return {"kernel": "mlp_kernel", "bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / BF16_PEAK_TFLOPS, "traffic": None,
            "flop_per_launch": n_cand * MLP_FLOP_PER_POSE, "ms_per_launch": mlp_ms,
            "frac_vs_measured_mfma": ach / meas, "measured_mfma_tflops": ceil,
            "note": "MLP time = prediction (trunk + MLP) minus the trunk alone, HIP events, first 4 maps"}


def e1_sweep(nbt, ctx, s_gs=(5, 50, 100, 200), n_ps=(100, 250, 500, 750, 1000), oracle_max_s=60.0,
             oracle_n_ps=None, emit=None):
    """Stand-in for the paper's runtime sweep (Sec. V, online capabilities): N_P perspectives
    sampled in the 1 m ball around the PoI (Eq. 1), endpoint grid spacing s_G * s_Vox,
    s_Vox = 1 cm.  GPU: end-to-end (pose upload, kernels, IG download) and kernel-only;
    CPU: the single-threaded oracle (within oracle_max_s, only for N_P in oracle_n_ps when
    given).  Returns the rows; emit(row) is called for each as it is measured."""
    import math
    import numpy as np
    import torch
    import oracle
    from workloads import poses_ball, scene_tabletop
    sc = scene_tabletop(n=320, voxel=0.01, n_objects=120, seed=22588 + 7000)
    poi = np.asarray(sc.extra["object_tops"][0], np.float64)
    m = nbt.Map(ctx, sc.P, sc.voxel, sc.origin)
    spent = 0.0
    rows = []
    for s_g in s_gs:
        cam = nbt.camera_from_grid(math.radians(75.0), math.radians(65.0), 1.5, 0.01, s_g)
        for n_p in n_ps:
            poses = poses_ball(poi, 1.0, n_p, seed=22588 + 7000 + n_p)
            stream = torch.cuda.current_stream()
            dp = torch.from_numpy(poses).cuda()
            kern = _timed(lambda: nbt.eval_viewpoints(m, cam, dp, want_steps=False), 10, stream)

            def end_to_end():
                d = torch.from_numpy(poses).cuda()
                ig, _ = nbt.eval_viewpoints(m, cam, d, want_steps=False)
                return ig.cpu()

            end_to_end()
            t0 = time.perf_counter()
            for _ in range(10):
                end_to_end()
            e2e = (time.perf_counter() - t0) * 100.0
            row = {"s_G": s_g, "N_P": n_p, "rays_per_perspective": cam.width * cam.height,
                   "gpu_kernel_ms": kern, "gpu_end_to_end_ms": e2e}
            if spent < oracle_max_s and (oracle_n_ps is None or n_p in oracle_n_ps):
                t0 = time.perf_counter()
                oracle.eval_viewpoints(sc, (cam.width, cam.height, cam.tan_half_fov_h, cam.tan_half_fov_v,
                                            cam.range), poses)
                dt = time.perf_counter() - t0
                spent += dt
                row["cpu_oracle_ms"] = dt * 1e3
            rows.append(row)
            if emit:
                emit(row)
    m.close()
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="waves,tile_w_log2,tiles_per_wave,xcd_remap,pipeline_depth")
    ap.add_argument("--layout", choices=("linear", "column4", "column2", "column8"), default=None,
                    help="map storage order (default: the library's)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the trajectory and batched measurements")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the memory-probe ceilings (stream, gather) and the fractions against them")
    ap.add_argument("--only", choices=("trajectories", "batched", "surrogate", "surrogate_tabletop", "insert",
                                       "top_k", "ceilings"), default=None,
                    help="only run one of the extra workloads (one JSON object)")
    ap.add_argument("--e1-sweep", action="store_true",
                    help="only run the N_P x s_G runtime sweep at 1 cm voxels (one JSON object per line)")
    ap.add_argument("--fingerprint", action="store_true",
                    help="print the source fingerprint the counters summary must carry and exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (scale for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} (WORLD_SIZE={world}) is not supported: "
              "the IG evaluation shards by perspective with no exchange, and this build runs on a "
              "single MI355X.", file=sys.stderr)
        sys.exit(2)

    if args.fingerprint:
        print(kernel_fingerprint())
        return

    # the oracle's other workloads run in a child process on one core while the GPU is
    # measured (started before anything here touches the GPU)
    other_cpu = None
    if not (args.no_cpu_baseline or args.only or args.e1_sweep or args.calibrate_copy):
        other_cpu = start_other_baselines()

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

    if args.e1_sweep:
        e1_sweep(nbt, nbt.Context(0), emit=lambda row: print(json.dumps(row), flush=True))
        return
    if args.only:
        cx = nbt.Context(0)
        run = {"trajectories": lambda: extra_trajectories(nbt, cx, reps=3),
               "batched": lambda: extra_batch(nbt, cx, reps=5),
               "surrogate": lambda: extra_surrogate(nbt, cx),
               "surrogate_tabletop": lambda: extra_surrogate(nbt, cx, family="cfg2", n_maps=4),
               "insert": lambda: extra_insert(nbt, cx, reps=5),
               "top_k": lambda: extra_top_k(nbt, cx),
               "ceilings": lambda: measure_ceilings(nbt, cx)}[args.only]
        print(json.dumps({args.only: run()}), flush=True)
        return

    t_gen = time.perf_counter()
    w = make_config(2)
    scene, cam, poses = w.maps[0], w.camera, w.poses[0]
    _log(f"workload generated in {time.perf_counter() - t_gen:.1f} s: map {scene.P.shape}, "
         f"{poses.shape[0]} perspectives, {cam.width}x{cam.height} rays")

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = nbt.Context(0)
    if args.layout:
        ctx.set_map_layout(nbt.LAYOUT_NAMES.index(args.layout))
    if args.launch:
        ctx.set_launch(*[int(v) for v in args.launch.split(",")])
    prob = torch.from_numpy(scene.P).cuda()
    m = nbt.Map(ctx, prob, scene.voxel, scene.origin)
    dposes = torch.from_numpy(poses).cuda()
    n = poses.shape[0]
    ig = torch.empty(n, dtype=torch.float32, device="cuda")
    steps = torch.empty(n, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    tuned = None
    untuned = None
    if not args.layout and not args.launch:
        # the library's defaults first, so that the line states what the tuner buys
        untuned = {"map_layout": nbt.LAYOUT_NAMES[m.info()["layout"]], "launch": ctx.get_launch(),
                   "kernel_ms": _timed(lambda: nbt.eval_viewpoints(m, cam, dposes, ig_out=ig, want_steps=False),
                                       5, stream)}
        # untimed set-up: the library picks the map's storage order and the launch shape
        t_tune = time.perf_counter()
        launch, layout, tune_ms = nbt.autotune_map(m, cam, dposes, ig_out=ig)
        tuned = {"layout": nbt.LAYOUT_NAMES[layout], "launch": launch, "ms": tune_ms,
                 "seconds": time.perf_counter() - t_tune}
        _log(f"autotuned: {tuned}")

    def step():
        m.update(prob)
        nbt.eval_viewpoints(m, cam, dposes, ig_out=ig, want_steps=False)

    # The voxel-step count (for the roofline) comes from one untimed call that
    # asks for it; the timed launches return IG only, as a planner calls them.
    m.update(prob)
    nbt.eval_viewpoints(m, cam, dposes, ig_out=ig, steps_out=steps)
    ig_counted = ig.clone()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    m.check()
    if not torch.equal(ig, ig_counted):
        raise RuntimeError("IG differs between the counting and the non-counting launch")

    ceilings = None
    if not args.no_ceilings:
        _log("measuring the memory ceilings ...")
        ceilings = measure_ceilings(nbt, ctx)

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        m.update(prob)
        e1.record(stream)
        nbt.eval_viewpoints(m, cam, dposes, ig_out=ig, want_steps=False)
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
            "map_layout": nbt.LAYOUT_NAMES[m.info()["layout"]],
            "tuned_by": "nbt_ig_autotune_map (untimed set-up)" if tuned else "command line",
        },
        "rays_per_s": rays * args.steps / wall,
        "voxel_steps_per_s": total_steps * args.steps / wall,
        "voxel_steps_per_step": total_steps,
        "kernel_ms": {"encode_map": enc_ms, "ig_viewpoints": ray_ms},
        "untuned": untuned,
        "tuner_speedup": untuned["kernel_ms"] / ray_ms if untuned else None,
        "roofline": {
            "kernel": "ig_viewpoints_kernel",
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_gb_per_launch": alg_bytes / 1e9,
        },
    }
    shape = launch_key(nbt.LAYOUT_NAMES[m.info()["layout"]], ctx.get_launch())
    counters = measured_counters(shape)
    if counters is not None:
        # HBM-side bytes of one launch from the committed rocprofv3 passes (FETCH_SIZE and
        # WRITE_SIZE scaled by a copy kernel of known size), as a rate over this run's launch
        # time so that it compares with `achieved`.
        traffic_b = float(counters["traffic bytes per launch"])
        result["roofline"]["traffic"] = traffic_b / (ray_ms * 1e-3) / 1e9
        result["roofline"]["traffic_gb_per_launch"] = traffic_b / 1e9
        result["binding_unit"] = {
            "unit": "TA (vector-memory address path) and VALU issue",
            "ta_busy_frac": float(counters["TA busy fraction"]),
            "valu_instr_per_cu_cycle": float(counters["VALU per CU-cycle"]),
            "tcp_accesses_per_gather": float(counters["L1 accesses per gather"]),
            "source": COUNTERS_PROFILE,
            "launch": shape,
        }
    else:
        result["roofline"]["traffic_note"] = (f"no committed counters for these sources and this map order and "
                                              f"launch shape ({shape})")
    if ceilings:
        result["roofline"]["levels"] = level_fractions(total_steps / (ray_ms * 1e-3), int(m.info()["device_bytes"]),
                                                       ceilings)
        result["memory_ceilings"] = ceilings
    if not args.no_extras:
        cx = nbt.Context(0)            # default settings, untouched by the main line's tuning
        _log("measuring trajectory IG (256^3 map, 4096 trajectories x 24 poses) ...")
        result["trajectories"] = extra_trajectories(nbt, cx, reps=3, ceilings=ceilings)
        _log("measuring the batched launch (64 maps, uneven perspective counts) ...")
        result["batched"] = extra_batch(nbt, cx, reps=5, ceilings=ceilings)
        _log("measuring the surrogate (64^3 sphere maps, 65,536 candidates) ...")
        result["surrogate"] = extra_surrogate(nbt, cx)
        _log("measuring the surrogate on 256^3 table-top maps (65,536 candidates) ...")
        result["surrogate_tabletop"] = extra_surrogate(nbt, cx, family="cfg2", n_maps=4)
        _log("measuring the map update by depth insertion ...")
        result["insert"] = extra_insert(nbt, cx, reps=5)
        _log("measuring next-best-view selection (top-k) ...")
        result["top_k"] = extra_top_k(nbt, cx)
        _log("measuring the runtime sweep at 1 cm voxels (compact) ...")
        result["e1_sweep"] = {
            "workload": "320^3 table-top map at 1 cm, N_P start points in the 1 m ball around an object top "
                        "(Eq. 1), endpoint grid s_G x 1 cm on the far plane (75x65 deg, 1.5 m); GPU kernel and "
                        "end-to-end (pose upload, evaluation, IG download) ms; the oracle at N_P = 100",
            "rows": e1_sweep(nbt, cx, n_ps=(100, 500, 1000), oracle_n_ps=(100,), oracle_max_s=5.0)}
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle baseline ...")
        result["cpu_baseline"] = cpu_baseline(scene, cam, poses, args.cpu_seconds)
        result["cpu_baseline"]["other_workloads"] = finish_other_baselines(other_cpu)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
