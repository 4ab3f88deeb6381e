"""Host-side pieces of bench.py: the counter-summary lookup that feeds
roofline.traffic, and the CPU oracle baseline."""
import hashlib
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_is_reported_only_while_the_source_hash_matches(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source v1\n")
    good = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "traffic.md"
    prof.write_text(f"traffic_bytes_per_launch k_x: 1.5e6\nsource_sha256 k.hip: {good}\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_x", "k.hip") == pytest.approx(1.5e6)
    assert bench.measured_traffic("k_y", "k.hip") is None          # kernel not listed
    src.write_bytes(b"kernel source v2\n")                          # kernel changed since
    assert bench.measured_traffic("k_x", "k.hip") is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("k_x", "k.hip") is None


def test_cpu_baseline_reports_cores_sample_and_single_core():
    from paper_2510_12011_amd import inputs
    spec = inputs.tiny_cube(n=6, n_steps=8)
    out = bench.cpu_baseline(spec, 8)
    assert out["kind"] == "oracle" and out["unit"] == "DOF*steps/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "first 8 steps" in out["sample"]
    assert out["single_core"]["value"] > 0
    assert "one thread" in out["single_core"]["sample"]
