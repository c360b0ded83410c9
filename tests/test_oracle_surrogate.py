"""Pins of the surrogate's float64 reference (no GPU)."""

import numpy as np
import pytest

from oracle import surrogate as S


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1 + 2 ** -9, 1 + 3 * 2 ** -9, 0.1, -2.5, 65504.0, 2 ** -130], np.float32)
    got = S.bf16_round(vals)
    # 1+2^-9 is halfway between 1 and 1+2^-7: ties to even -> 1; 1+3*2^-9 rounds up
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1 + 2 ** -7
    assert got[3] == 0.10009765625 and got[4] == -2.5 and got[5] == 65536.0
    assert got[6] == np.float32(2 ** -130)           # exactly representable subnormal


def _conv_bruteforce(x, w, b):
    ci, s = x.shape[0], x.shape[1]
    so = s // 2
    out = np.zeros((w.shape[0], so, so, so))
    for co in range(w.shape[0]):
        for z in range(so):
            for y in range(so):
                for xx in range(so):
                    acc = b[co]
                    for c in range(ci):
                        for dz in range(3):
                            for dy in range(3):
                                for dx in range(3):
                                    iz, iy, ix = 2 * z + dz - 1, 2 * y + dy - 1, 2 * xx + dx - 1
                                    if 0 <= iz < s and 0 <= iy < s and 0 <= ix < s:
                                        acc += w[co, c, dz, dy, dx] * x[c, iz, iy, ix]
                    out[co, z, y, xx] = acc
    return out


def test_conv_matches_bruteforce_definition():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 6, 6, 6))
    w = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    assert np.allclose(S.conv3d_s2(x, w, b), _conv_bruteforce(x, w, b), atol=1e-12)


def test_conv_centre_tap_is_strided_subsampling():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 8, 8))
    w = np.zeros((2, 2, 3, 3, 3))
    w[0, 0, 1, 1, 1] = 1.0
    w[1, 1, 1, 1, 1] = 2.0
    out = S.conv3d_s2(x, w, np.zeros(2))
    assert np.array_equal(out[0], x[0, ::2, ::2, ::2]) and np.array_equal(out[1], 2 * x[1, ::2, ::2, ::2])


def test_patch_counts_by_hand():
    # 8^3 map, voxel 0.1, origin 0: extent 1.6 -> cells of 0.05 -> f = max(1, round(0.5)) = 1?
    # use extent 6.4 -> cell 0.2 = 2 voxels, f = 2; PoI at (0.4, 0.4, 0.4) -> i0 = 4 - 32 = -28
    P = np.full((8, 8, 8), 0.2, np.float32)
    P[3, 5, 6] = 0.9          # occupied voxel (x=6, y=5, z=3)
    P[0, 0, 0] = 0.5          # unknown voxel
    p = S.extract_patch(P, 0.1, (0, 0, 0), (0.4, 0.4, 0.4), 6.4)
    f, i0 = S.patch_geometry((0.4, 0.4, 0.4), 6.4, 0.1, (0, 0, 0))
    assert f == 2 and i0 == [-28, -28, -28]
    # voxel (6,5,3) -> cell ((6+28)//2, (5+28)//2, (3+28)//2) = (17, 16, 15) in x, y, z
    assert p[0, 15, 16, 17] == 1 / 8 and p[0].sum() == 1 / 8
    assert p[1, 14, 14, 14] == 1 / 8 and p[1].sum() == 1 / 8


def test_patch_fully_inside_equals_block_means():
    rng = np.random.default_rng(3)
    P = rng.choice(np.array([0.2, 0.5, 0.9], np.float32), size=(64, 64, 64))
    p = S.extract_patch(P, 0.05, (0, 0, 0), (1.6, 1.6, 1.6), 3.2)      # f = 2, covers the map
    occ = (P > 0.5).reshape(32, 2, 32, 2, 32, 2).mean(axis=(1, 3, 5))
    unk = (P == np.float32(0.5)).reshape(32, 2, 32, 2, 32, 2).mean(axis=(1, 3, 5))
    assert np.array_equal(p[0], occ) and np.array_equal(p[1], unk)


def _random_params(rng, scale=0.1):
    return {name: rng.normal(size=shape) * scale for name, shape in S.weight_shapes()}


def test_pack_unpack_roundtrip():
    rng = np.random.default_rng(4)
    params = _random_params(rng)
    blob = S.pack_weights(params, 3.2, 0.8, 0.25, 40.0)
    got, meta = S.unpack_weights(blob)
    assert meta == {"extent": np.float32(3.2), "dist_mean": np.float32(0.8),
                    "dist_scale": np.float32(0.25), "out_scale": np.float32(40.0)}
    for name, _ in S.weight_shapes():
        assert np.array_equal(got[name], params[name].astype(np.float32).astype(np.float64))
    with pytest.raises(ValueError):
        S.unpack_weights(blob[:-4])


def test_head_reproduces_distance_with_hand_set_weights():
    """fc1 passes the normalised distance (plus a bias keeping it positive), fc2 copies it,
    fc3 reads it out: the prediction is an affine function of |t - PoI| only."""
    params = {name: np.zeros(shape) for name, shape in S.weight_shapes()}
    params["fc1.w"][0, S.N_FEAT + 3] = 1.0
    params["fc1.b"][0] = 10.0
    params["fc2.w"][0, 0] = 1.0
    params["fc3.w"][0] = 1.0
    params["fc3.b"][0] = -10.0
    meta = {"dist_mean": 0.8, "dist_scale": 0.25, "out_scale": 2.0}
    poi = np.array([1.0, 2.0, 3.0])
    poses = np.zeros((3, 12))
    poses[:, 9:] = poi + np.array([[0.5, 0, 0], [0, 1.0, 0], [0, 0, -1.3]])
    y = S.head(params, meta, np.zeros(S.N_FEAT), poses, poi, emulate_bf16=False)
    assert np.allclose(y, 2.0 * (np.array([0.5, 1.0, 1.3]) - 0.8) / 0.25)


def test_top_k_tie_break():
    v = np.array([1.0, 3.0, 2.0, 3.0, 0.5, 2.0])
    assert list(S.top_k(v, 4)) == [1, 3, 2, 5]


def test_library_blob_writer_matches_reference_layout():
    """The package's writer and the reference's reader agree on the documented layout."""
    from paper_2503_22588_amd.surrogate_blob import write_blob
    rng = np.random.default_rng(9)
    params = _random_params(rng)
    blob = write_blob(params, 3.2, 0.85, 0.26, 41.5)
    assert blob == S.pack_weights(params, 3.2, 0.85, 0.26, 41.5)
    got, meta = S.unpack_weights(blob)
    assert np.array_equal(got["fc2.w"], params["fc2.w"].astype(np.float32).astype(np.float64))


def _torch_forward_f64(params, meta, patch, poses, poi):
    """The surrogate's forward pass written with torch's own float64 CPU layers
    (conv3d with stride 2 and zero padding 1, ReLU, flatten, linear): a second,
    independent definition of the architecture documented in the blob format."""
    import torch
    import torch.nn.functional as F
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    x = t(patch)[None]                                      # [1, 2, 32, 32, 32] = (N, C, z, y, x)
    for k in range(4):
        x = F.relu(F.conv3d(x, t(params[f"conv{k + 1}.w"]), t(params[f"conv{k + 1}.b"]), stride=2, padding=1))
    feats = x.reshape(-1)                                   # channel-major, then z, y, x
    v = t(np.asarray(poses, np.float64).reshape(-1, 12)[:, 9:12]) - t(np.asarray(poi, np.float64))
    d = torch.linalg.vector_norm(v, dim=1, keepdim=True)
    inp = torch.cat([feats.expand(v.shape[0], -1), v / d, (d - meta["dist_mean"]) / meta["dist_scale"]], dim=1)
    h1 = F.relu(F.linear(inp, t(params["fc1.w"]), t(params["fc1.b"])))
    h2 = F.relu(F.linear(h1, t(params["fc2.w"]), t(params["fc2.b"])))
    y = F.linear(h2, t(params["fc3.w"])[None], t(params["fc3.b"]))[:, 0]
    return feats.numpy(), (meta["out_scale"] * y).numpy()


def _lively_params(rng):
    """Random weights scaled per layer so that activations neither die nor explode (about
    half of every layer's ReLUs active), rounded to float32 as the blob stores them."""
    params = {}
    for k, (ci, co) in enumerate(S.LAYERS):
        fan = ci * 27
        params[f"conv{k + 1}.w"] = rng.normal(size=(co, ci, 3, 3, 3)) * np.sqrt(2.0 / fan)
        params[f"conv{k + 1}.b"] = rng.normal(size=co) * 0.05
    params["fc1.w"] = rng.normal(size=(S.HIDDEN, S.N_IN)) * np.sqrt(2.0 / S.N_IN)
    params["fc1.b"] = rng.normal(size=S.HIDDEN) * 0.05
    params["fc2.w"] = rng.normal(size=(S.HIDDEN, S.HIDDEN)) * np.sqrt(2.0 / S.HIDDEN)
    params["fc2.b"] = rng.normal(size=S.HIDDEN) * 0.05
    params["fc3.w"] = rng.normal(size=S.HIDDEN) * np.sqrt(1.0 / S.HIDDEN)
    params["fc3.b"] = rng.normal(size=1) * 0.05
    return {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}


def test_float64_forward_equals_torch_layers():
    """predict(emulate_bf16=False) against torch's conv3d / linear in float64 on the CPU: pins
    the layer chaining, the ReLU after every layer but the last, the flatten order
    c*8 + z*4 + y*2 + x and the fc1 block that multiplies non-zero trunk features."""
    rng = np.random.default_rng(21)
    params = _lively_params(rng)
    blob = S.pack_weights(params, 3.2, 0.85, 0.26, 41.5)
    P = rng.choice(np.array([0.2, 0.5, 0.9], np.float32), p=[0.5, 0.4, 0.1], size=(64, 64, 64))
    poi = np.array([1.63, 1.58, 1.61])
    poses = np.zeros((300, 12), np.float32)
    dirs = rng.normal(size=(300, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    poses[:, 9:] = poi + dirs * rng.uniform(0.4, 1.3, size=(300, 1))
    got = S.predict(blob, P, 0.05, (0, 0, 0), poi, poses, emulate_bf16=False)
    prm, meta = S.unpack_weights(blob)
    patch = S.extract_patch(P, 0.05, (0, 0, 0), poi, meta["extent"])
    feats_ref, ref = _torch_forward_f64(prm, meta, patch, poses, poi)
    feats = S.trunk(prm, patch, emulate_bf16=False)
    # the features are alive (not a zero vector that would hide the fc1 block) and varied
    assert np.count_nonzero(feats_ref) > 100 and np.std(ref) > 1e-3 * np.abs(ref).max()
    np.testing.assert_allclose(feats, feats_ref, rtol=1e-12, atol=1e-12 * np.abs(feats_ref).max())
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_float64_forward_flatten_order_is_channel_then_z_y_x():
    """A single conv4 channel and one fc1 weight per feature position: the prediction reads
    exactly the feature that torch's flatten puts at c*8 + z*4 + y*2 + x."""
    rng = np.random.default_rng(22)
    params = _lively_params(rng)
    patch = rng.uniform(0.0, 1.0, size=(2, 32, 32, 32))
    feats = S.trunk(params, patch, emulate_bf16=False).reshape(64, 2, 2, 2)
    for c, z, y, x in [(0, 0, 0, 1), (3, 1, 0, 0), (17, 0, 1, 0), (63, 1, 1, 1)]:
        p = {k: v.copy() for k, v in params.items()}
        p["fc1.w"][:] = 0.0
        p["fc1.b"][:] = 0.0
        p["fc1.w"][0, c * 8 + z * 4 + y * 2 + x] = 1.0
        p["fc2.w"][:] = 0.0
        p["fc2.b"][:] = 0.0
        p["fc2.w"][0, 0] = 1.0
        p["fc3.w"][:] = 0.0
        p["fc3.w"][0] = 1.0
        p["fc3.b"][:] = 0.0
        meta = {"dist_mean": 0.8, "dist_scale": 0.25, "out_scale": 1.0}
        poses = np.zeros((1, 12))
        poses[0, 9:] = (1.0, 0.0, 0.0)
        y_pred = S.head(p, meta, feats.reshape(-1), poses, np.zeros(3), emulate_bf16=False)
        assert y_pred[0] == max(feats[c, z, y, x], 0.0)
