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
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(str(prof), "k_x", "k.hip") == pytest.approx(1.5e6)
    assert bench.measured_traffic(str(prof), "k_y", "k.hip") is None   # kernel not listed
    src.write_bytes(b"kernel source v2\n")                          # kernel changed since
    assert bench.measured_traffic(str(prof), "k_x", "k.hip") is None
    assert bench.measured_traffic(str(tmp_path / "missing.md"), "k_x", "k.hip") is None


def test_cpu_baseline_reports_cores_sample_and_single_core():
    from paper_2510_12011_amd import inputs
    spec = inputs.tiny_cube(n=6, n_steps=8)
    out = bench.cpu_baseline(spec, 8)
    assert out["kind"] == "oracle" and out["unit"] == "DOF*steps/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "first 8 steps" in out["sample"]
    assert out["single_core"]["value"] > 0
    assert "one thread" in out["single_core"]["sample"]


def test_cpu_baseline_window_starts_from_the_checkpoint():
    """The window baseline runs the oracle from a given state (the
    benchmark's checkpoint) and reports the host's CPU model."""
    from oracle import orc
    from paper_2510_12011_amd import inputs
    spec = inputs.tiny_cube(n=6, n_steps=30)
    o = orc.Oracle(spec)
    o.steps(20)
    st = o.state
    ck = dict(V=st.V.copy(), Vprev=st.Vprev.copy(), u=st.u.copy(), lat=st.lat.copy(),
              lrt=st.lrt.copy(), step=st.k)
    out = bench.cpu_baseline_window(spec, ck, 8)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] >= 1
    assert "window" in out["sample"] and out["cpu_model"] in out["sample"]
    assert out["single_core"]["value"] > 0
