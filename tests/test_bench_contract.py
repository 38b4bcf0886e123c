"""Host-side checks of the benchmark's contract (no GPU): more than one GPU is
refused with a message before anything touches a device, and the bottom
kernel's HBM bytes are taken from the committed rocprofv3 summary only while
that summary describes the current kernel sources and the benchmark's
workload."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def _source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_13793_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def test_traffic_only_from_a_summary_of_the_current_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.md"
    good.write_text("# k_bottom\n\ntraffic_bytes_per_launch: 123456789\n"
                    f"kernel_source_sha256: {_source_hash()}\n")
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 123456789\nkernel_source_sha256: " + "0" * 64 + "\n")
    monkeypatch.setattr(bench, "PROFILE", str(good))
    assert bench.profiled_traffic(256, 6, "fp64") == 123456789
    # other workloads have no committed byte counts
    assert bench.profiled_traffic(512, 6, "fp64") is None
    assert bench.profiled_traffic(256, 6, "fp32") is None
    monkeypatch.setattr(bench, "PROFILE", str(stale))
    assert bench.profiled_traffic(256, 6, "fp64") is None
