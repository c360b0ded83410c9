"""Train the learned IG surrogate on labels from the library's own exact raycaster.

Offline tool (not on any timed path).  Data: seeded scenes of the config-1
family (64^3 maps, 5 cm voxels, random occupied balls, free/unknown halves
split by a random plane through the map centre = the PoI), candidate camera
centres uniform in volume in the 0.4-1.3 m shell around the PoI looking at it,
labels g_P from nbt_ig_eval_viewpoints with the config-1 camera (64x48 rays,
60x45 deg, 2 m).  Inputs: the library's patch (nbt_ig_extract_patch) rounded
to BF16 as inference sees it, plus direction and distance.  The network is
the architecture the inference kernels implement; the result is written as
the packed weights blob nbt_ig_surrogate_create reads.

    python -m paper_2503_22588_amd.train_surrogate --out weights.nbts
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EXTENT = 3.2
R_IN, R_OUT = 0.4, 1.3
DIST_MEAN = 0.5 * (R_IN + R_OUT)
DIST_SCALE = (R_OUT - R_IN) / np.sqrt(12.0)


def _scene(seed):
    from workloads import scene_spheres
    n_sph = 10 + seed % 31                       # 10..40 balls: vary the clutter
    sc = scene_spheres(n=64, voxel=0.05, n_spheres=n_sph, seed=seed)
    return sc.P, np.asarray(sc.poi, np.float32)


def _poses(poi, n, seed):
    from workloads import poses_shell
    return poses_shell(poi.astype(np.float64), R_IN, R_OUT, n, seed)


def generate_scenes(seeds):
    """Scene grids, generated in this process before the GPU is used."""
    t0 = time.time()
    scenes = [_scene(sd) for sd in seeds]
    print(f"  {len(seeds)} scenes generated in {time.time() - t0:.1f} s", flush=True)
    return scenes


def build_dataset(nbt, ctx, cam, seeds, scenes, per_scene):
    """Patches [S,2,32,32,32] (BF16-rounded), poses [S,P,12], exact IG [S,P]."""
    import torch
    patches, poses, labels = [], [], []
    for k, (P, poi) in enumerate(scenes):
        m = nbt.Map(ctx, P, 0.05, (0.0, 0.0, 0.0))
        ps = _poses(poi, per_scene, seeds[k] + 500)
        dp = torch.from_numpy(ps).cuda()
        ig, _ = nbt.eval_viewpoints(m, cam, dp)
        patch = nbt.extract_patch(m, poi, EXTENT)
        torch.cuda.synchronize()
        patches.append(patch.to(torch.bfloat16).float().cpu())
        poses.append(torch.from_numpy(ps))
        labels.append(ig.cpu())
        m.close()
    return torch.stack(patches), torch.stack(poses), torch.stack(labels), [s[1] for s in scenes]


def make_model():
    import torch.nn as nn

    class Net(nn.Module):
        def __init__(self):
            super().__init__()
            chans = [2, 16, 32, 64, 64]
            self.convs = nn.ModuleList([nn.Conv3d(chans[i], chans[i + 1], 3, stride=2, padding=1) for i in range(4)])
            self.fc1 = nn.Linear(516, 256)
            self.fc2 = nn.Linear(256, 256)
            self.fc3 = nn.Linear(256, 1)

        def trunk(self, x):
            import torch
            for c in self.convs:
                x = torch.relu(c(x))
            return x.flatten(1)

        def head(self, feat, dirs):
            import torch
            h = torch.relu(self.fc1(torch.cat([feat, dirs], dim=-1)))
            h = torch.relu(self.fc2(h))
            return self.fc3(h).squeeze(-1)

    return Net()


def direction_inputs(poses, poi):
    import torch
    v = poses[..., 9:12] - poi[:, None, :]
    d = torch.linalg.norm(v, dim=-1, keepdim=True)
    return torch.cat([v / d.clamp_min(1e-9), (d - DIST_MEAN) / DIST_SCALE], dim=-1)


def export(model, out_scale, path):
    from paper_2503_22588_amd.surrogate_blob import write_blob
    params = {}
    for k, c in enumerate(model.convs):
        params[f"conv{k + 1}.w"] = c.weight.detach().cpu().double().numpy()
        params[f"conv{k + 1}.b"] = c.bias.detach().cpu().double().numpy()
    for name in ("fc1", "fc2", "fc3"):
        lin = getattr(model, name)
        params[f"{name}.w"] = lin.weight.detach().cpu().double().numpy().reshape(-1) if name == "fc3" else \
            lin.weight.detach().cpu().double().numpy()
        params[f"{name}.b"] = lin.bias.detach().cpu().double().numpy()
    blob = write_blob(params, EXTENT, DIST_MEAN, DIST_SCALE, out_scale)
    with open(path, "wb") as f:
        f.write(blob)
    return blob


def _spearman(a, b):
    ra = np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(np.float64)
    rb = np.argsort(np.argsort(b, kind="stable"), kind="stable").astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float(np.sum(ra * rb) / np.sqrt(np.sum(ra * ra) * np.sum(rb * rb)))


def evaluate(nbt, ctx, cam, blob, seeds, n_cand=65536, k_rescores=(64, 256, 1024), k=10):
    """Held-out quality over n_cand candidates per map: top-k agreement of the surrogate's
    selection with the exact top-k and the exact IG of its best pick relative to the true
    best, for each rescoring budget; plus the normalised mean absolute error and the rank
    correlation of the raw predictions.  (A relative error per candidate is not reported:
    candidates inside an occupied ball have near-zero exact IG and dominate such a mean.)"""
    import torch
    sur = nbt.Surrogate(ctx, blob)
    agree = {kr: [] for kr in k_rescores}
    best = {kr: [] for kr in k_rescores}
    nmae, rho = [], []
    for sd in seeds:
        P, poi = _scene(sd)
        m = nbt.Map(ctx, P, 0.05, (0.0, 0.0, 0.0))
        dp = torch.from_numpy(_poses(poi, n_cand, sd + 500)).cuda()
        exact, _ = nbt.eval_viewpoints(m, cam, dp)
        pred = sur.predict(m, poi, dp)
        torch.cuda.synchronize()
        ex = exact.cpu().numpy().astype(np.float64)
        pr = pred.cpu().numpy().astype(np.float64)
        top = set(np.lexsort((np.arange(n_cand), -ex))[:k].tolist())
        for kr in k_rescores:
            idx, ig = sur.select(m, cam, poi, dp, k_rescore=kr, k=k)
            torch.cuda.synchronize()
            agree[kr].append(len(top & set(int(v) for v in idx.cpu().numpy())) / k)
            best[kr].append(float(ig.cpu().numpy()[0]) / float(ex.max()))
        nmae.append(float(np.mean(np.abs(pr - ex)) / np.mean(ex)))
        rho.append(_spearman(pr, ex))
        m.close()
    sur.close()
    return {"maps": len(seeds), "candidates": n_cand, "k": k,
            "top_k_agreement": {str(kr): float(np.mean(v)) for kr, v in agree.items()},
            "best_ig_ratio": {str(kr): float(np.mean(v)) for kr, v in best.items()},
            "worst_best_ig_ratio": {str(kr): float(np.min(v)) for kr, v in best.items()},
            "per_map_agreement": {str(kr): v for kr, v in agree.items()},
            "nmae": float(np.mean(nmae)), "spearman": float(np.mean(rho))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="surrogate.nbts")
    ap.add_argument("--scenes", type=int, default=12288)
    ap.add_argument("--per-scene", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed-base", type=int, default=22588 + 5000)
    ap.add_argument("--listwise", type=float, default=1.0, help="weight of the listwise ranking term")
    ap.add_argument("--tau", type=float, default=0.05, help="softmax temperature of the listwise term")
    ap.add_argument("--log", default=None)
    ap.add_argument("--eval-maps", type=int, default=16, help="held-out maps for the quality report")
    args = ap.parse_args()

    seeds = [args.seed_base + i for i in range(args.scenes)]
    print("building training set ...", flush=True)
    scenes = generate_scenes(seeds)

    import torch
    import paper_2503_22588_amd as nbt
    from workloads.configs import CAM1

    torch.manual_seed(0)
    torch.cuda.init()
    ctx = nbt.Context(0)
    X, Pz, Y, pois = build_dataset(nbt, ctx, CAM1, seeds, scenes, args.per_scene)
    poi_t = torch.from_numpy(np.stack(pois))
    out_scale = float(Y.mean())
    print(f"  {X.shape[0]} scenes x {Y.shape[1]} poses, IG mean {out_scale:.3f} std {float(Y.std()):.3f}",
          flush=True)
    dev = "cuda"
    X, Pz, Y, poi_t = X.to(dev), Pz.to(dev), (Y / out_scale).to(dev), poi_t.to(dev)
    D = direction_inputs(Pz, poi_t)
    n_val = max(64, X.shape[0] // 32)
    tr, va = slice(n_val, X.shape[0]), slice(0, n_val)
    model = make_model().to(dev)
    opt = torch.optim.AdamW(model.parameters(), lr=args.lr, weight_decay=1e-5)
    steps_per_epoch = max(1, (X.shape[0] - n_val) // args.batch_scenes)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=args.lr, total_steps=args.epochs * steps_per_epoch)
    log = []
    t0 = time.time()
    for ep in range(args.epochs):
        model.train()
        perm = torch.randperm(X.shape[0] - n_val, device=dev) + n_val
        tot = 0.0
        for b in range(steps_per_epoch):
            idx = perm[b * args.batch_scenes:(b + 1) * args.batch_scenes]
            feat = model.trunk(X[idx])                                  # [B, 512]
            f = feat[:, None, :].expand(-1, Y.shape[1], -1)
            pred = model.head(f, D[idx])
            y = Y[idx]
            loss = torch.nn.functional.smooth_l1_loss(pred, y, beta=0.05)
            # pairwise ranking within each scene, half of the pairs anchored at the scene's
            # best 5 %: selection only needs the order near the top to be right
            B, Pn = y.shape
            n_top = max(1, Pn // 20)
            top_i = torch.topk(y, n_top, dim=1).indices
            pi = torch.cat([torch.gather(top_i, 1, torch.randint(0, n_top, (B, 64), device=dev)),
                            torch.randint(0, Pn, (B, 64), device=dev)], dim=1)
            pj = torch.randint(0, Pn, (B, 128), device=dev)
            dy = torch.gather(y, 1, pi) - torch.gather(y, 1, pj)
            dp = torch.gather(pred, 1, pi) - torch.gather(pred, 1, pj)
            rank = torch.relu(0.01 - torch.sign(dy) * dp)[dy.abs() > 0.01].mean()
            loss = loss + 0.5 * torch.nan_to_num(rank)
            if args.listwise > 0:
                # listwise term: cross-entropy between the softmax of the labels and of the
                # predictions over each scene's candidates, which weighs the top of the list
                tgt = torch.softmax(y / args.tau, dim=1)
                loss = loss - args.listwise * (tgt * torch.log_softmax(pred / args.tau, dim=1)).sum(1).mean()
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            sched.step()
            tot += float(loss.detach())
        model.eval()
        with torch.no_grad():
            pv = torch.cat([model.head(model.trunk(X[va][i:i + 16])[:, None, :].expand(-1, Y.shape[1], -1),
                                       D[va][i:i + 16]) for i in range(0, n_val, 16)])
            yv = Y[va]
            nmae = float((pv - yv).abs().mean() / yv.mean())
            nmae_const = float((yv - Y[tr].mean()).abs().mean() / yv.mean())
            rho = float(np.mean([_spearman(pv[i].cpu().numpy(), yv[i].cpu().numpy()) for i in range(n_val)]))
        log.append({"epoch": ep, "loss": tot / steps_per_epoch, "val_nmae": nmae, "val_spearman": rho,
                    "t": time.time() - t0})
        print(f"epoch {ep:3d} loss {tot / steps_per_epoch:.5f} val nmae {nmae:.4f} (constant {nmae_const:.4f}) "
              f"spearman {rho:.3f} ({time.time() - t0:.0f} s)", flush=True)
    blob = export(model.cpu(), out_scale, args.out)
    print(f"wrote {args.out} ({len(blob)} bytes)", flush=True)
    held = [args.seed_base + 100000 + i for i in range(args.eval_maps)]
    quality = evaluate(nbt, ctx, CAM1, blob, held) if args.eval_maps else None
    print(f"held-out quality: {quality}", flush=True)
    if args.log:
        json.dump({"args": vars(args), "out_scale": out_scale, "epochs": log, "held_out": quality},
                  open(args.log, "w"), indent=1)


if __name__ == "__main__":
    main()
