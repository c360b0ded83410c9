"""Writer of the surrogate weights blob that nbt_ig_surrogate_create reads.

Layout (little-endian): b"NBTS", uint32 version 1, float32 extent, dist_mean,
dist_scale, out_scale, two reserved uint32; then float32 arrays in this order:
conv1..conv4 weight [cout][cin][3][3][3] and bias [cout] (channels 2-16-32-64-64),
fc1 weight [256][516] and bias, fc2 weight [256][256] and bias, fc3 weight [256]
and bias [1].
"""

from __future__ import annotations

import struct

import numpy as np

CONV_CHANNELS = (2, 16, 32, 64, 64)


def blob_layout():
    out = []
    for k in range(4):
        ci, co = CONV_CHANNELS[k], CONV_CHANNELS[k + 1]
        out += [(f"conv{k + 1}.w", (co, ci, 3, 3, 3)), (f"conv{k + 1}.b", (co,))]
    out += [("fc1.w", (256, 516)), ("fc1.b", (256,)), ("fc2.w", (256, 256)), ("fc2.b", (256,)),
            ("fc3.w", (256,)), ("fc3.b", (1,))]
    return out


def write_blob(params: dict, extent: float, dist_mean: float, dist_scale: float, out_scale: float) -> bytes:
    parts = [b"NBTS", struct.pack("<I", 1), struct.pack("<4f", extent, dist_mean, dist_scale, out_scale),
             struct.pack("<2I", 0, 0)]
    for name, shape in blob_layout():
        a = np.asarray(params[name], dtype="<f4")
        if a.size != int(np.prod(shape)):
            raise ValueError(f"{name}: expected {shape}, got {a.shape}")
        parts.append(np.ascontiguousarray(a.reshape(shape)).tobytes())
    return b"".join(parts)
