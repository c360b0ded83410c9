"""The C ABI library loads and exports every declared entry point (no GPU needed)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbt_ig.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbt_ig_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for required in ("nbt_ig_create_map", "nbt_ig_eval_viewpoints", "nbt_ig_trace_rays",
                     "nbt_ig_ctx_create", "nbt_ig_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2503_22588_amd as nbt
    lib = C.CDLL(nbt.binding.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_host_only_helpers():
    import math
    import paper_2503_22588_amd as nbt
    b = nbt.binding
    assert b.abi_version() == 1
    assert b.status_string(b.EINVAL) == "invalid argument"
    # paper's operating point: s_Vox = 1 cm, s_G = 100 -> 1 m endpoint spacing on the far plane
    cam = nbt.camera_from_grid(math.radians(90), math.radians(60), 2.0, 0.01, 100)
    assert (cam.width, cam.height) == (5, 3)        # 2*2*tan45/1 = 4 -> 5; 2*2*tan30 = 2.31 -> 3
    assert cam.tan_half_fov_h == pytest.approx(1.0)
    with pytest.raises(nbt.NbtError) as e:
        nbt.camera_from_grid(0.0, 1.0, 2.0, 0.01, 100)
    assert e.value.status == b.EINVAL


def test_insertion_defaults_are_the_oracles():
    """The library's default log-odds parameters carry the same binary32 bits as the oracle's
    (log(p/(1-p)) of 0.7, 0.4, 0.1192, 0.971), and a NULL map needs no workspace."""
    import numpy as np
    import oracle
    import paper_2503_22588_amd as nbt
    lib = np.array(nbt.insert_default_params(), np.float32)
    ref = np.array(oracle.DEFAULT_INSERT_PARAMS, np.float32)
    assert np.array_equal(lib.view(np.int32), ref.view(np.int32))
    assert nbt.binding._lib.nbt_ig_insert_workspace_words(None) == 0


def test_context_creation_reports_missing_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the gpu tests")
    import paper_2503_22588_amd as nbt
    with pytest.raises(nbt.NbtError) as e:
        nbt.Context(0)
    assert e.value.status in (nbt.binding.EDEVICE, nbt.binding.EINVAL)


def test_binding_constants_match_the_header():
    """Every numeric constant the binding mirrors (status codes, ray end reasons, voxel states,
    map layouts) has the header's value."""
    import paper_2503_22588_amd as nbt
    text = open(HEADER).read()
    values = {name: int(v) for name, v in re.findall(r"\bNBT_IG_([A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    checked = 0
    for name, v in values.items():
        if hasattr(nbt.binding, name):
            assert getattr(nbt.binding, name) == v, name
            checked += 1
    for required in ("OK", "EINVAL", "RAY_HIT", "RAY_EXIT", "OCCUPIED", "LAYOUT_LINEAR", "LAYOUT_COLUMN4"):
        assert required in values and hasattr(nbt.binding, required), required
    assert checked >= 14


def test_noalloc_limit_matches_the_header():
    import paper_2503_22588_amd as nbt
    m = re.search(r"#define\s+NBT_IG_NOALLOC_MAX_VIEWPOINTS\s+(\d+)u?", open(HEADER).read())
    assert m and int(m.group(1)) == nbt.binding.NOALLOC_MAX_VIEWPOINTS


def test_probe_constants_match_the_header():
    import paper_2503_22588_amd as nbt
    text = open(HEADER).read()
    for name in ("PROBE_STREAM", "PROBE_GATHER", "PROBE_QUAD_GATHER", "PROBE_MFMA_16X16X32_BF16",
                 "PROBE_MFMA_32X32X16_BF16"):
        m = re.search(rf"#define\s+NBT_IG_{name}\s+(\d+)", text)
        assert m and int(m.group(1)) == getattr(nbt.binding, name), name
