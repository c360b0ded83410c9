"""Float64 reference of the learned IG surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate is not in the paper (its own cheap estimate of IG between
perspectives is the IDW interpolation of Eq. 3); it is the network this
project trains on IG labels of its own raycaster.  This module is the plain
definition of its forward pass, written from the architecture below, used to
check the BF16 MFMA kernels.  Rounding to bfloat16 happens at exactly the
points where the GPU stores bfloat16 (`emulate_bf16=True`); every sum is
taken in float64 with NumPy's tensordot/matmul as the only library steps.

Architecture (weights blob layout, little-endian float32 after a 32-byte header
"NBTS", version 1, extent, dist_mean, dist_scale, out_scale, 2 reserved words):
  patch   2 x 32^3: fraction of occupied / unknown voxels per cell of a cube of
          side `extent` around the PoI, snapped to the voxel grid
  conv1..conv4: 3^3 kernels, stride 2, zero padding 1, ReLU; channels
          2 -> 16 -> 32 -> 64 -> 64, spatial 32 -> 16 -> 8 -> 4 -> 2
          (weights [cout][cin][dz][dy][dx], bias [cout])
  features f = conv4 output flattened as c*8 + z*4 + y*2 + x  (512)
  input  [f, u_x, u_y, u_z, (|v| - dist_mean) / dist_scale]  (516),
          v = camera centre - PoI, u = v / |v|
  fc1 516 -> 256 ReLU, fc2 256 -> 256 ReLU, fc3 256 -> 1, times out_scale
"""

from __future__ import annotations

import struct

import numpy as np

MAGIC = b"NBTS"
GRID = 32
LAYERS = [(2, 16), (16, 32), (32, 64), (64, 64)]
HIDDEN = 256
N_FEAT = 512
N_IN = N_FEAT + 4


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even); returned as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = x32.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------ weights --

def weight_shapes():
    shapes = []
    for k, (ci, co) in enumerate(LAYERS):
        shapes += [(f"conv{k + 1}.w", (co, ci, 3, 3, 3)), (f"conv{k + 1}.b", (co,))]
    shapes += [("fc1.w", (HIDDEN, N_IN)), ("fc1.b", (HIDDEN,)), ("fc2.w", (HIDDEN, HIDDEN)),
               ("fc2.b", (HIDDEN,)), ("fc3.w", (HIDDEN,)), ("fc3.b", (1,))]
    return shapes


def pack_weights(params: dict, extent, dist_mean, dist_scale, out_scale) -> bytes:
    head = MAGIC + struct.pack("<I4f2I", 1, extent, dist_mean, dist_scale, out_scale, 0, 0)
    body = b"".join(np.ascontiguousarray(params[name], dtype="<f4").reshape(shape).tobytes()
                    for name, shape in weight_shapes())
    return head + body


def unpack_weights(blob: bytes):
    if blob[:4] != MAGIC:
        raise ValueError("not a surrogate weights blob")
    version, extent, dmean, dscale, oscale, _, _ = struct.unpack("<I4f2I", blob[4:32])
    if version != 1:
        raise ValueError("unsupported surrogate weights version")
    params, off = {}, 32
    for name, shape in weight_shapes():
        n = int(np.prod(shape))
        params[name] = np.frombuffer(blob, dtype="<f4", count=n, offset=off).reshape(shape).astype(np.float64)
        off += 4 * n
    if off != len(blob):
        raise ValueError("surrogate weights blob has the wrong size")
    meta = {"extent": extent, "dist_mean": dmean, "dist_scale": dscale, "out_scale": oscale}
    return params, meta


# ------------------------------------------------------------------ patch ----

def patch_geometry(poi, extent, voxel, origin):
    """Cells of f^3 voxels; cell c covers voxels [i0 + c f, i0 + (c+1) f) per axis."""
    f = max(1, int(np.floor(extent / (GRID * voxel) + 0.5)))
    i0 = [int(np.floor((float(poi[a]) - float(origin[a])) / voxel + 0.5)) - (GRID // 2) * f for a in range(3)]
    return f, i0


def extract_patch(P, voxel, origin, poi, extent, thresholds=(0.5, 0.5)):
    """Occupied and unknown fractions per cell [2, 32, 32, 32] (z, y, x); voxels
    outside the map count as neither."""
    P = np.asarray(P, dtype=np.float32)
    nz, ny, nx = P.shape
    occ = (P > np.float32(thresholds[0])).astype(np.float64)
    unk = (~(P > np.float32(thresholds[0])) & ~(P < np.float32(thresholds[1]))).astype(np.float64)
    f, (ix, iy, iz) = patch_geometry(poi, extent, voxel, origin)
    side = GRID * f
    out = np.zeros((2, GRID, GRID, GRID))
    for ch, src in enumerate((occ, unk)):
        block = np.zeros((side, side, side))
        zs, ys, xs = [max(0, -i) for i in (iz, iy, ix)]
        z0, y0, x0 = max(iz, 0), max(iy, 0), max(ix, 0)
        z1, y1, x1 = min(iz + side, nz), min(iy + side, ny), min(ix + side, nx)
        if z1 > z0 and y1 > y0 and x1 > x0:
            block[zs:zs + z1 - z0, ys:ys + y1 - y0, xs:xs + x1 - x0] = src[z0:z1, y0:y1, x0:x1]
        out[ch] = block.reshape(GRID, f, GRID, f, GRID, f).sum(axis=(1, 3, 5)) / float(f ** 3)
    return out


# ------------------------------------------------------------------ network --

def conv3d_s2(x, w, b):
    """out[co,z,y,x] = b[co] + sum_{ci,dz,dy,dx} w[co,ci,dz,dy,dx] xpad[ci, 2z+dz, 2y+dy, 2x+dx]."""
    ci, s = x.shape[0], x.shape[1]
    so = s // 2
    xp = np.zeros((ci, s + 2, s + 2, s + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.zeros((w.shape[0], so, so, so)) + b[:, None, None, None]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                tap = xp[:, dz:dz + 2 * so:2, dy:dy + 2 * so:2, dx:dx + 2 * so:2]
                out += np.tensordot(w[:, :, dz, dy, dx], tap, axes=([1], [0]))
    return out


def trunk(params, patch, emulate_bf16=True):
    """Conv layers on one patch -> 512 features (float64)."""
    r = bf16_round if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    x = r(patch)
    for k in range(len(LAYERS)):
        w = r(params[f"conv{k + 1}.w"])
        x = np.maximum(conv3d_s2(x, w, params[f"conv{k + 1}.b"]), 0.0)
        x = r(x)
    return x.reshape(-1)


def direction_inputs(poses, poi, dist_mean, dist_scale):
    v = np.asarray(poses, dtype=np.float64).reshape(-1, 12)[:, 9:12] - np.asarray(poi, dtype=np.float64)
    d = np.linalg.norm(v, axis=1)
    u = v / np.where(d > 0, d, 1.0)[:, None]
    return np.concatenate([u, ((d - dist_mean) / dist_scale)[:, None]], axis=1)


def head(params, meta, feats, poses, poi, emulate_bf16=True):
    """MLP on [features, direction, distance] for every pose -> predicted IG."""
    r = bf16_round if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    w1 = params["fc1.w"]
    dirs = direction_inputs(poses, poi, meta["dist_mean"], meta["dist_scale"])
    h1 = r(feats)[None, :] @ r(w1[:, :N_FEAT]).T + dirs @ w1[:, N_FEAT:].T + params["fc1.b"][None, :]
    h1 = r(np.maximum(h1, 0.0))
    h2 = np.maximum(h1 @ r(params["fc2.w"]).T + params["fc2.b"][None, :], 0.0)
    y = h2 @ params["fc3.w"] + params["fc3.b"][0]
    return meta["out_scale"] * y


def predict(blob, P, voxel, origin, poi, poses, thresholds=(0.5, 0.5), emulate_bf16=True):
    params, meta = unpack_weights(blob)
    patch = extract_patch(P, voxel, origin, poi, meta["extent"], thresholds)
    return head(params, meta, trunk(params, patch, emulate_bf16), poses, poi, emulate_bf16)


def top_k(values, k):
    """Indices of the k largest values, ties broken by the lower index."""
    v = np.asarray(values, dtype=np.float64)
    order = sorted(range(len(v)), key=lambda i: (-v[i], i))
    return np.array(order[:k], dtype=np.int64)
