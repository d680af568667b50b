"""Host logic of bench.py (no GPU): the one-GPU contract, the class-tile count
behind the launch floor, the byte model's unit counts and the roofline
arithmetic."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("h,w", [(1080, 1920), (2160, 3840), (321, 481), (1, 1), (5, 200),
                                 (12, 192), (13, 193)])
def test_pixel_tiles_counts_the_class0_tiles(h, w):
    # brute force: class-0 pixels are those with x % 3 == 0 and y % 3 == 0; a
    # tile holds 64 x 4 of them in class coordinates
    tiles = {(x // 3 // 64, y // 3 // 4) for y in range(0, h, 3) for x in range(0, w, 3)}
    assert bench.pixel_tiles(h, w) == len(tiles)


@pytest.mark.parametrize("uw,uh", [(1, 1), (2, 5), (7, 7), (481, 321), (60, 34)])
def test_class_units_partition_the_unit_grid(uw, uh):
    counts = [bench.class_units(uw, uh, c) for c in range(9)]
    assert sum(counts) == uw * uh
    for c in range(9):
        brute = sum(1 for y in range(uh) for x in range(uw) if x % 3 == c % 3 and y % 3 == c // 3)
        assert counts[c] == brute


def test_units_of_rounds_up():
    assert bench.units_of(1080, 1920, 3) == (240, 135)
    assert bench.units_of(321, 481, 2) == (121, 81)
    assert bench.units_of(1, 1, 4) == (1, 1)


def test_structural_bytes_are_the_label_plane_and_the_class_bins():
    # side 4 of 1080p, class 0: 480 x 270 labels of 4 B, 160 x 90 blocks of 16 pixels
    assert bench.structural_phase_bytes(1080, 1920, 2, 0) == 4.0 * 480 * 270 + 160 * 90 * 16


def test_roofline_fractions_follow_from_bytes_and_time():
    prof = {"bytes_per_launch": 274537.0, "structural_bytes_per_launch": 1947600.0,
            "levels": [{"side": 1, "pixels": 10, "beta": 0.1}]}
    r = bench.roofline("k", prof, 6.788, traffic=3933000)
    assert r["achieved"] == pytest.approx(274537.0 / 6.788e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert r["structural_frac"] == pytest.approx(1947600.0 / 6.788e-6 / 1e9 / 8000.0, rel=1e-3)
    assert r["traffic_over_algorithmic"] == pytest.approx(3933000 / 274537.0, abs=0.01)
    assert "pixels" not in r["per_level"][0]
    skipped = bench.roofline("k", None, 6.788)
    assert skipped["frac"] is None and skipped["note"] == "byte pass skipped"


def test_measured_traffic_is_used_only_for_the_kernels_it_was_taken_on(tmp_path):
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"kernel_source_sha256": bench.kernel_source_hash(),
                                "traffic_bytes_per_launch": 123}))
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"kernel_source_sha256": "0" * 64,
                                 "traffic_bytes_per_launch": 123}))
    assert bench.measured_traffic(str(good)) == 123
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "absent.json")) is None
