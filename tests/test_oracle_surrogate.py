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
