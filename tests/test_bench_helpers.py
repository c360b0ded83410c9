"""The arithmetic of bench.py's roofline objects (CPU only): the algorithmic rate against the
HBM peak, the choice of the measured ceiling by the map's size, the MLP's FLOP count, and a
non-positive MLP time giving no rate, and the committed counters applying only to the launch
shape they were taken with."""

import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


CEIL = {"1MiB": {"stream_gbs": 25000.0, "gather_words_per_s": 2.5e11, "quad_gather_words_per_s": 1e12},
        "64MiB": {"stream_gbs": 7000.0, "gather_words_per_s": 6e10, "quad_gather_words_per_s": 2.4e11},
        "1GiB": {"stream_gbs": 6400.0, "gather_words_per_s": 5.6e10, "quad_gather_words_per_s": 2.2e11}}


def test_roofline_of_walk():
    r = bench.roofline_of("k", 1.5e12, 70 << 20, CEIL)
    assert r["achieved"] == pytest.approx(6000.0)            # 4 B per step
    assert r["frac"] == pytest.approx(6000.0 / 8000.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["traffic"] is None
    lv = r["levels"]
    assert lv["ceiling_working_set"] == "64MiB" and lv["level"].startswith("Infinity Cache")
    assert lv["frac_vs_stream"] == pytest.approx(6000.0 / 7000.0)
    assert lv["frac_vs_gather"] == pytest.approx(1.5e12 / 6e10)


@pytest.mark.parametrize("mib,label", [(1, "1MiB"), (4, "1MiB"), (5, "64MiB"), (192, "64MiB"), (193, "1GiB")])
def test_level_by_map_size(mib, label):
    assert bench.level_fractions(1e12, mib << 20, CEIL)["ceiling_working_set"] == label
    assert bench.level_fractions(1e12, mib << 20, None) is None


def test_mlp_flops_and_guard(monkeypatch):
    # fc2 256x256, the per-pose part of fc1 (256 x 4 inputs) and fc3 (256): 2 FLOP per product
    assert bench.MLP_FLOP_PER_POSE == 2 * (256 * 256 + 256 * 4 + 256)
    monkeypatch.setattr(bench, "measure_mfma_ceiling", lambda nbt, ctx: {"32x32x16_bf16_2wave_tflops": 2400.0})
    r = bench.mlp_roofline(None, None, 65536, 0.0133)
    assert r["achieved"] == pytest.approx(65536 * bench.MLP_FLOP_PER_POSE / 13.3e-6 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 2500.0)
    assert r["frac_vs_measured_mfma"] == pytest.approx(r["achieved"] / 2400.0)
    for bad in (0.0, -0.001, float("nan")):
        r = bench.mlp_roofline(None, None, 65536, bad)
        assert r["achieved"] is None and r["frac"] is None


def test_counters_only_for_their_launch_shape():
    """The committed counters are used only for the sources, map order and launch shape they
    were taken with."""
    key = bench.launch_key("column4", {"waves_per_group": 2, "tile_w_log2": 3, "tiles_per_wave": 4,
                                       "xcd_remap": 0, "pipeline_depth": 8})
    assert key == "column4 2,3,4,0,8"
    vals = bench.measured_counters()
    if vals is None:
        pytest.skip("the committed counters were taken for other sources")
    assert "launch" in vals and "fingerprint" in vals
    assert bench.measured_counters(vals["launch"]) == vals
    assert bench.measured_counters("linear 1,0,1,0,1") is None


def test_counters_blocks_per_launch_shape(tmp_path, monkeypatch):
    """A summary may hold one block of values per launch shape; each shape gets its own."""
    fp = bench.kernel_fingerprint()
    (tmp_path / "c.md").write_text(f"text\n\n- fingerprint: `{fp}`\n\n- launch: column4 1,3,4,0,8\n"
                                   "- traffic bytes per launch: 100\n- TA busy fraction: 0.9\n\n"
                                   "- launch: column4 1,3,2,0,8\n- traffic bytes per launch: 200\n"
                                   "- TA busy fraction: 0.8\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "COUNTERS_PROFILE", "c.md")
    monkeypatch.setattr(bench, "kernel_fingerprint", lambda: fp)
    a = bench.measured_counters("column4 1,3,4,0,8")
    b = bench.measured_counters("column4 1,3,2,0,8")
    assert a["traffic bytes per launch"] == "100" and a["TA busy fraction"] == "0.9"
    assert b["traffic bytes per launch"] == "200" and b["TA busy fraction"] == "0.8"
    assert a["fingerprint"] == fp == b["fingerprint"]
    assert bench.measured_counters() == a
    assert bench.measured_counters("column4 2,3,4,0,8") is None
    monkeypatch.setattr(bench, "kernel_fingerprint", lambda: "other")
    assert bench.measured_counters("column4 1,3,4,0,8") is None
