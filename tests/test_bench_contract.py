"""Host-side checks of bench.py's contract (no GPU).

* More than one GPU is refused with a message and exit status 2, before
  anything touches a device.
* The HBM traffic of the dominant kernel is taken from a committed counter
  summary only while the kernel sources hash to the value stored in it.
"""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a run that did not happen


def test_traffic_is_read_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_w_traffic.md").write_text("# traffic\n\nsource_sha256: abc123\ntraffic_bytes_per_launch: 2.5e8\n"
                                         "| table | row |\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "abc123")
    assert bench.measured_traffic("w", "k") == 2.5e8
    assert bench.measured_traffic("other", "k") is None  # no summary for this workload
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "def456")
    assert bench.measured_traffic("w", "k") is None  # the kernel changed since the counters were taken


@pytest.mark.parametrize("name", ["step_c2_traffic.md", "step_c4_traffic.md"])
def test_committed_summary_names_a_hash_of_the_right_form(name):
    path = os.path.join(ROOT, "profiles", name)
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", " ", "#", "`")):
                k, _, v = line.partition(":")
                kv[k.strip()] = v.strip()
    assert len(kv["source_sha256"]) == 64 and int(kv["source_sha256"], 16) >= 0
    assert float(kv["traffic_bytes_per_launch"]) > 0
