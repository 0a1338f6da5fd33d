"""Host-side checks of bench.py's measurement plumbing (no GPU): the one-GPU guard, and the HBM
traffic figure, which is read from the committed counter summary only while that summary names
the current near-kernel sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_hash_covers_the_near_kernel_sources():
    names = sorted(os.path.basename(f) for f in bench.KERNEL_SOURCES)
    assert names == ["k_near.hip", "spm_internal.h"]
    assert all(os.path.exists(f) for f in bench.KERNEL_SOURCES)
    h = bench.kernel_hash()
    assert len(h) == 64 and h == bench.kernel_hash()


def test_traffic_summary_matches_the_sources():
    """The committed summary carries the hash of the sources it was measured on; the bench reports its
    bytes per launch only while that hash matches (it is null otherwise)."""
    t = bench.measured_traffic()
    assert t is not None, "the traffic summary was taken on other near-kernel sources"
    assert 2.0e6 < t < 1.0e8   # between the algorithmic 2.05 MB and a gross re-read


def test_traffic_is_null_for_other_sources(tmp_path, monkeypatch):
    other = tmp_path / "k_near.hip"
    other.write_text("// other sources\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(other)])
    assert bench.measured_traffic() is None


def test_traffic_is_null_without_a_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None
