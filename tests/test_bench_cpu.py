"""Host logic of bench.py: the measured HBM traffic is reported only while the
kernel source and the tuner cache are the ones the counters were taken with."""

import hashlib

import bench


def _setup(tmp_path, src=b"kernel v1", tuned=b'{"a": [1]}', value=123456):
    k = tmp_path / "raycast.hip"
    t = tmp_path / "tuned.json"
    c = tmp_path / "counters.md"
    k.write_bytes(src)
    t.write_bytes(tuned)
    c.write_text(f"# counters\nkernel source sha256: {hashlib.sha256(src).hexdigest()}\n"
                 f"tuner cache sha256: {hashlib.sha256(tuned).hexdigest()}\n\n"
                 f"traffic_bytes_per_launch: {value}\n")
    return k, t, c


def test_traffic_reported_when_hashes_match(tmp_path, monkeypatch):
    k, t, c = _setup(tmp_path)
    monkeypatch.setattr(bench, "KERNEL_SRC", str(k))
    monkeypatch.setattr(bench, "TUNED", str(t))
    monkeypatch.setattr(bench, "COUNTERS", str(c))
    assert bench.measured_traffic() == 123456


def test_traffic_withheld_after_a_kernel_or_cache_change(tmp_path, monkeypatch):
    k, t, c = _setup(tmp_path)
    monkeypatch.setattr(bench, "KERNEL_SRC", str(k))
    monkeypatch.setattr(bench, "TUNED", str(t))
    monkeypatch.setattr(bench, "COUNTERS", str(c))
    k.write_bytes(b"kernel v2")
    assert bench.measured_traffic() is None
    k.write_bytes(b"kernel v1")
    t.write_bytes(b'{"a": [2]}')
    assert bench.measured_traffic() is None
    t.write_bytes(b'{"a": [1]}')
    assert bench.measured_traffic() == 123456
    c.write_text(c.read_text().replace("tuner cache sha256", "tuner sha"))
    assert bench.measured_traffic() is None          # a summary without the cache hash is stale
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None

