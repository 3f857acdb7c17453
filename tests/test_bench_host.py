"""Host logic of bench.py that runs without a GPU: the one-GPU guard and the
gate that reports counter traffic only for the kernel sources it was
measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_is_machine_readable(monkeypatch):
    """The committed counter summary carries the per-launch and per-step
    bytes and the hash of the sources they were taken on."""
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: _file_hash())
    vals = bench._traffic_values()
    assert vals is not None
    assert vals["kernel"] == "bfs_rev"
    assert int(vals["traffic_bytes_per_launch"]) > 0
    assert int(vals["step_traffic_bytes"]) > int(vals["traffic_bytes_per_launch"])
    assert bench.measured_traffic("bfs_rev") == float(vals["traffic_bytes_per_launch"])
    assert bench.measured_step_traffic() == float(vals["step_traffic_bytes"])
    assert bench.measured_traffic("push") is None  # counters of the dominant kernel only


def test_traffic_is_withheld_once_the_sources_change(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench._traffic_values() is None
    assert bench.measured_traffic("bfs_rev") is None
    assert bench.measured_step_traffic() is None


def test_source_hash_covers_the_kernel_sources(tmp_path, monkeypatch):
    a = tmp_path / "a.h"
    b = tmp_path / "b.hip"
    a.write_text("x")
    b.write_text("y")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a), str(b)])
    h0 = bench.kernel_source_hash()
    b.write_text("y ")
    assert bench.kernel_source_hash() != h0
    assert len(h0) == 64


def _file_hash():
    with open(bench.TRAFFIC_FILE) as f:
        for line in f:
            if line.strip().startswith("- kernel_source_sha256:"):
                return line.split(":", 1)[1].strip()
    pytest.fail("no source hash in the counter summary")
