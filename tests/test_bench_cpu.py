"""Host logic of bench.py: the measured HBM traffic and L2 hit rates are
reported only while the kernel source and the launch's tile shape are the
ones the counters were taken with; frame timings that cannot bracket the render, or
that put the frame above the HBM peak, are refused."""

import hashlib

import numpy as np
import pytest

import bench


SHAPE = (4, 1, 1, 16, 4, 0)


def _setup(tmp_path, src=b"kernel v1", value=123456):
    k = tmp_path / "raycast.hip"
    c = tmp_path / "counters.md"
    k.write_bytes(src)
    c.write_text(f"# counters\nkernel source sha256: {hashlib.sha256(src).hexdigest()}\n"
                 f"tile shape: 4,1,1,16,4,0\n\n"
                 f"| kernel | fetch |\n|---|---|\n| raycast_kernel | 1 |\n\n"
                 f"traffic_bytes_per_frame: {value}\n"
                 f"l2_hit_rate raycast_kernel: 0.75\nl2_hit_rate derive_kernel: 0.125\n")
    return k, c


def _patch(monkeypatch, k, c):
    monkeypatch.setattr(bench, "KERNEL_SRC", str(k))
    monkeypatch.setattr(bench, "COUNTERS", str(c))


def test_traffic_reported_when_hashes_match(tmp_path, monkeypatch):
    k, c = _setup(tmp_path)
    _patch(monkeypatch, k, c)
    assert bench.measured_traffic(SHAPE) == 123456
    assert bench.measured_l2_hit_rate(SHAPE) == {"raycast_kernel": 0.75, "derive_kernel": 0.125}


def test_traffic_withheld_after_a_kernel_or_shape_change(tmp_path, monkeypatch):
    k, c = _setup(tmp_path)
    _patch(monkeypatch, k, c)
    k.write_bytes(b"kernel v2")
    assert bench.measured_traffic(SHAPE) is None
    assert bench.measured_l2_hit_rate(SHAPE) is None
    k.write_bytes(b"kernel v1")
    assert bench.measured_traffic((8, 2, 1, 16, 4, 0)) is None        # another tile shape
    assert bench.measured_traffic(SHAPE) == 123456
    c.write_text(c.read_text().replace("tile shape", "shape"))
    assert bench.measured_traffic(SHAPE) is None          # a summary without the shape is stale
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.md"))
    assert bench.measured_traffic(SHAPE) is None


def test_rooflines_from_frame_and_kernel_times(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.md"))
    frame = np.array([0.2, 0.2, 0.2])
    hbm, alu = bench.rooflines(frame, 0.1, 514_035_936, 1.2e7)
    assert hbm["bound"] == "hbm" and hbm["unit"] == "GB/s"
    assert hbm["achieved"] == pytest.approx(514_035_936 / 0.2e-3 / 1e9, rel=1e-3)
    assert 0 < hbm["frac"] <= 1
    assert hbm["frame_ms_mean"] >= alu["kernel_avg_ms"]
    assert alu["peak"] == 157.3 and alu["frac"] == pytest.approx(alu["achieved"] / 157.3, abs=1e-4)


def test_frame_events_that_miss_the_render_are_refused(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.md"))
    # events on another stream time only the host enqueue: shorter than the kernel they contain
    with pytest.raises(RuntimeError, match="bracket"):
        bench.rooflines(np.array([0.0187, 0.02]), 0.1042, 514_035_936, 1.2e7)
    # a frame time that puts the algorithmic bytes above the HBM peak
    with pytest.raises(RuntimeError, match="peak"):
        bench.rooflines(np.array([0.05]), 0.04, 514_035_936, 1.2e7)


def test_oracle_view_samples_only_for_the_headline_size():
    ref = bench.oracle_view_samples(256, 1920, 1080, "f32")
    assert ref is not None and len(ref["samples"]) == 26
    assert all(s > 0 for s in ref["samples"])
    assert bench.oracle_view_samples(128, 1920, 1080, "f32") is None
    assert bench.oracle_view_samples(256, 1920, 1080, "f16") is None
