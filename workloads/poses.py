"""Seeded camera poses around a point of interest.

A pose is 12 float32 values: a row-major 3x3 rotation ``R`` (camera to world;
its columns are the camera x axis = image right, y axis = image down and z
axis = viewing direction) followed by the camera centre ``t`` in world
coordinates.  Perspectives look from their start point toward the point of
interest (Sec. III, perspective selection); the roll about the viewing axis
is fixed by keeping the camera x axis horizontal (world +Z is "up"), falling
back to world +Y when the view is within 0.8 degrees of vertical.  A camera
placed exactly at its target looks straight down.
"""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def look_at(positions, poi):
    """Poses at ``positions`` [N,3] whose z axis points at ``poi`` [3] (or [N,3])."""
    p = np.asarray(positions, dtype=np.float64).reshape(-1, 3)
    q = np.broadcast_to(np.asarray(poi, dtype=np.float64), p.shape)
    z = q - p
    nrm = np.linalg.norm(z, axis=1, keepdims=True)
    degenerate = nrm[:, 0] == 0
    nrm[degenerate] = 1.0
    z = z / nrm
    z[degenerate] = (0.0, 0.0, -1.0)          # no view vector: look straight down
    up = np.zeros_like(z)
    near_vertical = np.abs(z[:, 2]) > 0.9999
    up[~near_vertical, 2] = 1.0
    up[near_vertical, 1] = 1.0
    x = np.cross(z, up)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=2)            # columns are the camera axes
    out = np.empty((p.shape[0], 12), dtype=np.float32)
    out[:, :9] = R.reshape(-1, 9).astype(np.float32)
    out[:, 9:] = p.astype(np.float32)
    return out


def _unit_normals(rng, n):
    """Muller's method: normalised i.i.d. Gaussian vectors are uniform on the sphere."""
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def poses_sphere(poi, radius, n, seed):
    """``n`` perspectives uniform on the sphere of ``radius`` around ``poi``."""
    rng = _rng(seed)
    d = _unit_normals(rng, n)
    pos = np.asarray(poi, dtype=np.float64) + radius * d
    return look_at(pos, poi)


def poses_shell(poi, r_in, r_out, n, seed):
    """``n`` perspectives uniform in volume in the shell ``r_in <= r <= r_out``."""
    rng = _rng(seed)
    d = _unit_normals(rng, n)
    u = rng.uniform(0.0, 1.0, size=(n, 1))
    r = np.cbrt(r_in ** 3 + u * (r_out ** 3 - r_in ** 3))
    pos = np.asarray(poi, dtype=np.float64) + r * d
    return look_at(pos, poi)


def poses_ball(poi, r_s, n, seed):
    """Start points uniform in the ball of radius ``r_s`` around ``poi`` (Eq. 1).

    Directions come from Muller's method and the radius is ``r_s`` times the
    cube root of a U(0,1) draw; the point of interest is added as the offset.
    A start point that coincides with the point of interest gets the default
    orientation of ``look_at`` for a zero view vector.
    """
    rng = _rng(seed)
    d = _unit_normals(rng, n)
    xr = rng.uniform(0.0, 1.0, size=(n, 1))
    pos = np.asarray(poi, dtype=np.float64) + r_s * np.cbrt(xr) * d
    return look_at(pos, poi)


def _rotation(axis_angle):
    """Rodrigues' formula for a batch of rotation vectors [N,3] -> [N,3,3]."""
    th = np.linalg.norm(axis_angle, axis=1)
    k = np.zeros_like(axis_angle)
    nz = th > 0
    k[nz] = axis_angle[nz] / th[nz, None]
    K = np.zeros((len(th), 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -k[:, 2], k[:, 1]
    K[:, 1, 0], K[:, 1, 2] = k[:, 2], -k[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -k[:, 1], k[:, 0]
    s = np.sin(th)[:, None, None]
    c = np.cos(th)[:, None, None]
    return np.eye(3)[None] + s * K + (1 - c) * (K @ K)


def trajectories_walk(poi, n_traj, n_poses, seed, r_range=(0.6, 1.0), step=0.03,
                      heading_jitter_deg=15.0, rot_step_deg=4.0, rot_max_deg=15.0,
                      radial_jitter=0.01):
    """Smooth random-walk camera trajectories on a shell around ``poi``.

    Start: a Muller direction at a radius uniform in ``r_range``.  Each step
    turns a persistent tangent heading by up to +-15 degrees, moves 3 cm along
    it, jitters the radius and reflects it back into ``r_range``.  The view
    direction is look-at composed with an offset rotation that random-walks
    4 degrees per step and is reflected at 15 degrees.  Returns float32
    ``[n_traj, n_poses, 12]``.
    """
    rng = _rng(seed)
    poi = np.asarray(poi, dtype=np.float64)
    d = _unit_normals(rng, n_traj)
    r = rng.uniform(r_range[0], r_range[1], size=n_traj)
    h = np.cross(d, _unit_normals(rng, n_traj))
    h /= np.linalg.norm(h, axis=1, keepdims=True)
    omega = np.zeros((n_traj, 3))
    out = np.empty((n_traj, n_poses, 12), dtype=np.float32)
    rot_step = np.deg2rad(rot_step_deg)
    rot_max = np.deg2rad(rot_max_deg)
    for s in range(n_poses):
        pos = poi + r[:, None] * d
        base = look_at(pos, poi)
        Rb = base[:, :9].astype(np.float64).reshape(-1, 3, 3)
        R = Rb @ _rotation(omega)
        out[:, s, :9] = R.reshape(-1, 9).astype(np.float32)
        out[:, s, 9:] = pos.astype(np.float32)
        # heading: rotate about the radial direction by a bounded random angle
        ang = np.deg2rad(rng.uniform(-heading_jitter_deg, heading_jitter_deg, size=n_traj))
        h = (h * np.cos(ang)[:, None] + np.cross(d, h) * np.sin(ang)[:, None]
             + d * (np.sum(d * h, axis=1) * (1 - np.cos(ang)))[:, None])
        newp = pos + step * h
        r = r + rng.uniform(-radial_jitter, radial_jitter, size=n_traj)
        r = np.where(r < r_range[0], 2 * r_range[0] - r, r)
        r = np.where(r > r_range[1], 2 * r_range[1] - r, r)
        d = newp - poi
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        h = h - d * np.sum(h * d, axis=1, keepdims=True)
        h /= np.linalg.norm(h, axis=1, keepdims=True)
        # orientation offset: bounded random walk of the rotation vector
        omega = omega + rot_step * _unit_normals(rng, n_traj)
        mag = np.linalg.norm(omega, axis=1)
        over = mag > rot_max
        omega[over] *= ((2 * rot_max - mag[over]) / mag[over])[:, None]
    return out
