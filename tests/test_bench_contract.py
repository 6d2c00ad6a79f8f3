"""Host-side checks of bench.py's reporting: the traffic figure is only reported while the
counter summary matches the kernel source it was measured on."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_matches_committed_summary():
    text = open(bench.TRAFFIC_FILE).read()
    src = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    got = bench.measured_traffic()
    if f"source_sha256: {src}" in text:
        assert got is not None and got > 24.0 * 33718272  # at least the algorithmic bytes
    else:
        assert got is None


def test_traffic_is_null_for_a_changed_kernel(tmp_path, monkeypatch):
    changed = tmp_path / "kern.hip"
    changed.write_bytes(open(bench.KERNEL_SRC, "rb").read() + b"\n// edited\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(changed))
    assert bench.measured_traffic() is None


def test_traffic_is_null_without_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None
