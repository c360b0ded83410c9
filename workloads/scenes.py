"""Seeded voxel scenes (occupancy probability grids) for the benchmark configs.

Every grid is ``float32 P[nz][ny][nx]`` (x fastest), voxel ``(ix, iy, iz)``
spanning ``origin + voxel * [i, i + 1)`` on each axis.  Probabilities take the
three values a freshly built occupancy map would hold for the three voxel
states of the paper's map (Sec. III): occupied 0.9, free 0.2, unknown 0.5.
The generators only place geometry; they never compute gains.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

P_OCC = np.float32(0.9)
P_FREE = np.float32(0.2)
P_UNKNOWN = np.float32(0.5)


@dataclass
class SceneMap:
    """A dense occupancy-probability grid plus its placement in the world."""

    P: np.ndarray                 # float32 [nz, ny, nx]
    voxel: float                  # edge length in metres (float32-representable)
    origin: np.ndarray            # float32 [3], world position of voxel (0,0,0)'s min corner
    poi: np.ndarray               # float64 [3], point of interest used by the pose samplers
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.P.shape
        return nx, ny, nz

    def fractions(self):
        n = self.P.size
        return {
            "occupied": float(np.count_nonzero(self.P == P_OCC)) / n,
            "free": float(np.count_nonzero(self.P == P_FREE)) / n,
            "unknown": float(np.count_nonzero(self.P == P_UNKNOWN)) / n,
        }


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _dims3(n):
    if np.isscalar(n):
        return int(n), int(n), int(n)
    nx, ny, nz = (int(v) for v in n)
    return nx, ny, nz


def _centres(nx, ny, nz, voxel, origin):
    """Voxel-centre coordinates per axis (float64), broadcastable to [nz,ny,nx]."""
    xc = origin[0] + (np.arange(nx, dtype=np.float64) + 0.5) * voxel
    yc = origin[1] + (np.arange(ny, dtype=np.float64) + 0.5) * voxel
    zc = origin[2] + (np.arange(nz, dtype=np.float64) + 0.5) * voxel
    return xc[None, None, :], yc[None, :, None], zc[:, None, None]


def _paint_ball(P, occ_value, centre, radius, voxel, origin):
    """Set every voxel whose centre lies within ``radius`` of ``centre``."""
    nz, ny, nx = P.shape
    lo = np.floor((centre - radius - origin) / voxel).astype(np.int64)
    hi = np.floor((centre + radius - origin) / voxel).astype(np.int64) + 1
    lo = np.maximum(lo, 0)
    hi = np.minimum(hi, [nx, ny, nz])
    if np.any(hi <= lo):
        return 0
    xs = origin[0] + (np.arange(lo[0], hi[0]) + 0.5) * voxel
    ys = origin[1] + (np.arange(lo[1], hi[1]) + 0.5) * voxel
    zs = origin[2] + (np.arange(lo[2], hi[2]) + 0.5) * voxel
    d2 = ((xs[None, None, :] - centre[0]) ** 2 + (ys[None, :, None] - centre[1]) ** 2
          + (zs[:, None, None] - centre[2]) ** 2)
    inside = d2 <= radius * radius
    sub = P[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
    sub[inside] = occ_value
    return int(np.count_nonzero(inside))


def scene_spheres(n=64, voxel=0.05, n_spheres=20, seed=22588 + 1000,
                  r_range=(0.05, 0.15), origin=(0.0, 0.0, 0.0)) -> SceneMap:
    """Random occupied spheres in a box split into a free and an unknown half.

    The point of interest is the box centre.  A plane through it with a
    uniformly random normal separates free voxels (P = 0.2, positive side)
    from unknown ones (P = 0.5); ``n_spheres`` balls with centres uniform in
    the box and radii uniform in ``r_range`` are then painted occupied
    (P = 0.9, voxel centre inside the ball).
    """
    nx, ny, nz = _dims3(n)
    voxel = float(np.float32(voxel))
    origin = np.asarray(origin, dtype=np.float32)
    o64 = origin.astype(np.float64)
    ext = np.array([nx, ny, nz], dtype=np.float64) * voxel
    poi = o64 + ext / 2.0
    rng = _rng(seed)
    normal = rng.normal(size=3)
    normal /= np.linalg.norm(normal)
    xc, yc, zc = _centres(nx, ny, nz, voxel, o64)
    side = ((xc - poi[0]) * normal[0] + (yc - poi[1]) * normal[1]) + (zc - poi[2]) * normal[2]
    P = np.where(side > 0.0, P_FREE, P_UNKNOWN).astype(np.float32)
    centres = o64 + rng.uniform(0.0, 1.0, size=(n_spheres, 3)) * ext
    radii = rng.uniform(r_range[0], r_range[1], size=n_spheres)
    for c, r in zip(centres, radii):
        _paint_ball(P, P_OCC, c, r, voxel, o64)
    return SceneMap(P=P, voxel=voxel, origin=origin, poi=poi, name=f"spheres{nx}x{ny}x{nz}",
                    extra={"normal": normal, "sphere_centres": centres, "sphere_radii": radii})


def scene_uniform(n, value, voxel=0.05, origin=(0.0, 0.0, 0.0)) -> SceneMap:
    """A box filled with one probability value (analytic test scenes)."""
    nx, ny, nz = _dims3(n)
    voxel = float(np.float32(voxel))
    origin = np.asarray(origin, dtype=np.float32)
    P = np.full((nz, ny, nx), np.float32(value), dtype=np.float32)
    poi = origin.astype(np.float64) + np.array([nx, ny, nz]) * voxel / 2.0
    return SceneMap(P=P, voxel=voxel, origin=origin, poi=poi, name=f"uniform{value}")


def _tabletop_geometry(nx, ny, nz, voxel, rng, n_objects):
    """Boolean ground-truth geometry: a table slab plus boxes and cylinders."""
    ext = np.array([nx, ny, nz], dtype=np.float64) * voxel
    centre = ext / 2.0
    table_z = 0.4 * ext[2]                       # top surface height
    half = np.array([0.75, 0.5])                 # 1.5 m x 1.0 m top
    thick = 2 * voxel
    solid = np.zeros((nz, ny, nx), dtype=bool)
    xc, yc, zc = _centres(nx, ny, nz, voxel, np.zeros(3))

    def box(lo, hi):
        i0 = np.clip(np.floor(lo / voxel + 0.5).astype(int), 0, [nx, ny, nz])
        i1 = np.clip(np.floor(hi / voxel + 0.5).astype(int), 0, [nx, ny, nz])
        solid[i0[2]:i1[2], i0[1]:i1[1], i0[0]:i1[0]] = True

    box(np.array([centre[0] - half[0], centre[1] - half[1], table_z - thick]),
        np.array([centre[0] + half[0], centre[1] + half[1], table_z]))
    tops = []
    kinds = rng.integers(0, 2, size=n_objects)
    for k in kinds:
        px = centre[0] + rng.uniform(-half[0], half[0])
        py = centre[1] + rng.uniform(-half[1], half[1])
        if k == 0:
            sx, sy, sz = rng.uniform(0.02, 0.20, size=3)
            box(np.array([px - sx / 2, py - sy / 2, table_z]),
                np.array([px + sx / 2, py + sy / 2, table_z + sz]))
            tops.append((px, py, table_z + sz))
        else:
            r = rng.uniform(0.02, 0.08)
            h = rng.uniform(0.05, 0.30)
            i0 = np.clip(np.floor(np.array([px - r, py - r, table_z]) / voxel).astype(int), 0, [nx, ny, nz])
            i1 = np.clip(np.floor(np.array([px + r, py + r, table_z + h]) / voxel).astype(int) + 1,
                         0, [nx, ny, nz])
            sub_x = xc[:, :, i0[0]:i1[0]]
            sub_y = yc[:, i0[1]:i1[1], :]
            sub_z = zc[i0[2]:i1[2], :, :]
            inside = (((sub_x - px) ** 2 + (sub_y - py) ** 2) <= r * r) & (sub_z >= table_z) & \
                (sub_z <= table_z + h)
            solid[i0[2]:i1[2], i0[1]:i1[1], i0[0]:i1[0]] |= inside
            tops.append((px, py, table_z + h))
    return solid, np.array(tops), table_z, centre


def _seen_from(camera, solid, voxel, bin_size=0.004, splat=0.9, tol=0.5):
    """Voxels with a clear line of sight from ``camera`` (a z-buffer test).

    Object voxels are splatted into a depth buffer on the plane one metre
    below the camera (every object lies below it); a voxel is seen when its
    distance does not exceed the nearest object depth in its bin by more than
    half a voxel.  Voxels level with or above the camera are never occluded.
    """
    nz, ny, nx = solid.shape
    oz, oy, ox = np.nonzero(solid)
    objc = (np.stack([ox, oy, oz], axis=1) + 0.5) * voxel - camera
    below = objc[:, 2] < -voxel
    objc = objc[below]
    dist = np.linalg.norm(objc, axis=1)
    proj = objc[:, :2] / (-objc[:, 2:3])
    lim = np.abs(proj).max() + 0.05 if len(proj) else 1.0
    nb = int(np.ceil(2 * lim / bin_size)) + 1
    depth = np.full((nb, nb), np.inf)
    b = np.floor((proj + lim) / bin_size).astype(np.int64)
    # angular radius of a voxel seen at distance d, expressed in bins on the
    # projection plane (coarse upper bound: the projection stretches by 1/cos^2)
    rad = np.ceil((splat * voxel / dist) * (dist / -objc[:, 2]) ** 2 / bin_size).astype(np.int64)
    rmax = int(rad.max()) if len(rad) else 0
    for dy in range(-rmax, rmax + 1):
        for dx in range(-rmax, rmax + 1):
            sel = (dx * dx + dy * dy) <= rad * rad
            bx = np.clip(b[sel, 0] + dx, 0, nb - 1)
            by = np.clip(b[sel, 1] + dy, 0, nb - 1)
            np.minimum.at(depth, (by, bx), dist[sel])
    seen = np.ones(solid.shape, dtype=bool)
    xs = (np.arange(nx) + 0.5) * voxel - camera[0]
    ys = (np.arange(ny) + 0.5) * voxel - camera[1]
    for iz in range(nz):
        dz = (iz + 0.5) * voxel - camera[2]
        if dz >= -voxel:
            continue
        px = xs[None, :] / -dz
        py = ys[:, None] / -dz
        bx = np.floor((px + lim) / bin_size).astype(np.int64)
        by = np.floor((py + lim) / bin_size).astype(np.int64)
        inb = (bx >= 0) & (bx < nb) & (by >= 0) & (by < nb)
        d = np.sqrt(xs[None, :] ** 2 + ys[:, None] ** 2 + dz * dz)
        dep = np.full((ny, nx), np.inf)
        bxc = np.clip(bx, 0, nb - 1)
        byc = np.clip(by, 0, nb - 1)
        dep = np.where(inb, depth[byc, bxc], np.inf)
        seen[iz] = d <= dep + tol * voxel
    return seen


def scene_tabletop(n=256, voxel=0.02, n_objects=200, seed=22588 + 2000,
                   n_prior=3, origin=(0.0, 0.0, 0.0)) -> SceneMap:
    """Table-top clutter whose unknown region is the space hidden from prior views.

    A 1.5 m x 1.0 m table slab carries ``n_objects`` axis-aligned boxes (sides
    2-20 cm) and vertical cylinders (radius 2-8 cm, height 5-30 cm).  Three
    seeded prior camera centres 1.2-1.8 m above the table top decide what has
    been observed: seen object voxels are occupied (0.9), seen empty voxels
    free (0.2) and everything no prior camera could see is unknown (0.5).
    ``extra['object_tops']`` lists the top centre of every object (the
    candidate points of interest).
    """
    nx, ny, nz = _dims3(n)
    voxel = float(np.float32(voxel))
    origin = np.asarray(origin, dtype=np.float32)
    rng = _rng(seed)
    solid, tops, table_z, centre = _tabletop_geometry(nx, ny, nz, voxel, rng, n_objects)
    seen = np.zeros_like(solid)
    cams = []
    for _ in range(n_prior):
        az = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(0.3, 1.0)
        cam = np.array([centre[0] + rad * np.cos(az), centre[1] + rad * np.sin(az),
                        table_z + rng.uniform(1.2, 1.8)])
        cams.append(cam)
        seen |= _seen_from(cam, solid, voxel)
    P = np.full(solid.shape, P_UNKNOWN, dtype=np.float32)
    P[seen & ~solid] = P_FREE
    P[seen & solid] = P_OCC
    o64 = origin.astype(np.float64)
    tops_world = tops + o64
    return SceneMap(P=P, voxel=voxel, origin=origin, poi=tops_world[0], name=f"tabletop{nx}",
                    extra={"object_tops": tops_world, "prior_cameras": np.array(cams) + o64,
                           "table_z": table_z + o64[2]})


def batch_maps(n_maps=64, sizes=(64, 96, 128, 192, 256), voxel=0.05, cfg=3, base_spheres=20):
    """Independent sphere scenes of uneven size (sphere count scaled by volume)."""
    rng = _rng(22588 + 1000 * cfg + 999)
    picks = rng.integers(0, len(sizes), size=n_maps)
    maps = []
    for m, k in enumerate(picks):
        n = int(sizes[k])
        ns = int(round(base_spheres * (n / 64.0) ** 3))
        maps.append(scene_spheres(n=n, voxel=voxel, n_spheres=ns, seed=22588 + 1000 * cfg + m))
    return maps
