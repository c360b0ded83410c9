"""Synthetic depth images of the sphere scenes (inputs of the map update by depth insertion).

A depth camera measures, per pixel, the z-depth of the first surface along that pixel's ray.
The rays here are those of the endpoint grid (pixel (i, j) looks at the far-plane point
(u_i, v_j, range) in camera coordinates), and the surfaces are the analytic spheres that
``scene_spheres`` painted into its map, so the images describe the same world as the map
without reading the map.  Pure geometry in float64, rounded once to float32.
"""

from __future__ import annotations

import numpy as np


def depth_images(scene, camera, poses, invalid_frac=0.0, seed=0):
    """z-depth images [K, H, W] float32 of ``scene``'s spheres seen from ``poses`` [K, 12].

    Pixels that see no sphere get +inf (no return).  ``invalid_frac`` of the pixels, drawn
    with ``seed``, get 0 (no measurement), as depth cameras report dropped pixels.
    """
    centres = np.asarray(scene.extra["sphere_centres"], np.float64).reshape(-1, 3)
    radii = np.asarray(scene.extra["sphere_radii"], np.float64).reshape(-1)
    W, H, rng_m = int(camera.width), int(camera.height), float(np.float32(camera.range))
    th, tv = float(camera.tan_h), float(camera.tan_v)
    u = np.zeros(W) if W == 1 else rng_m * th * (2.0 * np.arange(W) - (W - 1)) / (W - 1)
    v = np.zeros(H) if H == 1 else rng_m * tv * (2.0 * np.arange(H) - (H - 1)) / (H - 1)
    cam_dirs = np.stack(np.broadcast_arrays(u[None, :], v[:, None], rng_m), -1)     # [H, W, 3]
    poses = np.asarray(poses, np.float64).reshape(-1, 12)
    out = np.full((poses.shape[0], H, W), np.inf)
    for k, p in enumerate(poses):
        R, c = p[:9].reshape(3, 3), p[9:]
        d = cam_dirs @ R.T                       # segment to the far-plane point, per pixel
        best = np.full((H, W), np.inf)
        for C, r in zip(centres, radii):
            oc = c - C
            a = np.einsum("hwk,hwk->hw", d, d)
            b = 2.0 * (d @ oc)
            cc = float(oc @ oc) - r * r
            disc = b * b - 4.0 * a * cc
            ok = disc >= 0.0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            t_near = (-b - sq) / (2.0 * a)
            t_far = (-b + sq) / (2.0 * a)
            t = np.where(t_near > 0.0, t_near, t_far)     # from inside a sphere: its far wall
            t = np.where(ok & (t > 0.0), t, np.inf)
            best = np.minimum(best, t)
        out[k] = best * rng_m                    # segment parameter -> z-depth in metres
    if invalid_frac > 0.0:
        drop = np.random.default_rng(seed).random(out.shape) < invalid_frac
        out[drop] = 0.0
    return out.astype(np.float32)
