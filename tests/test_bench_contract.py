"""Host-side checks of bench.py's reporting: the traffic figure is only reported while the
counter summary matches the kernel source it was measured on, and a request for several GPUs is
refused."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_matches_committed_summary():
    text = open(bench.TRAFFIC_FILE).read()
    src = hashlib.sha256(b"".join(open(f, "rb").read() for f in bench.KERNEL_SRCS)).hexdigest()
    got = bench.measured_traffic()
    if f"source_sha256: {src}" in text:
        assert got is not None and got > 24.0 * 33718272  # at least the algorithmic bytes
    else:
        assert got is None


def test_traffic_is_null_for_a_changed_kernel(tmp_path, monkeypatch):
    # an edit to either source the summary covers (the kernel or its shared header) voids it
    for k in range(len(bench.KERNEL_SRCS)):
        changed = tmp_path / f"src{k}"
        changed.write_bytes(open(bench.KERNEL_SRCS[k], "rb").read() + b"\n// edited\n")
        srcs = list(bench.KERNEL_SRCS)
        srcs[k] = str(changed)
        monkeypatch.setattr(bench, "KERNEL_SRCS", srcs)
        assert bench.measured_traffic() is None


def test_traffic_is_null_without_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    # the benchmark measures one GPU; asking for more ends with a message before any GPU work
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
