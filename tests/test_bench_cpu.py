"""Host-side pieces of bench.py: the one-GPU guard, the credited flop count
and the rule that a profiled traffic figure stands only while the kernel
sources it was measured on are unchanged."""
import hashlib
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_credited_covariance_flops():
    # Hermitian outer-product sum: n * pq (pq + 1) / 2 complex entries, each
    # one complex multiply-add (8 real flops) per snapshot
    for p, q, n in [(3, 8, 64), (3, 16, 200), (5, 24, 256)]:
        pq = p * q
        assert bench.scm_flops_per_pixel(p, q, n) == n * (pq * (pq + 1) // 2) * 8
    assert bench.scm_flops_per_pixel(3, 16, 200) == 1_881_600


def _profile(tmp_path, src_text, recorded_text):
    src = tmp_path / "kernel.hip"
    src.write_text(src_text)
    sha = hashlib.sha256(recorded_text.encode()).hexdigest()
    prof = tmp_path / "profile.md"
    prof.write_text(f"# summary\ntraffic_bytes_per_launch: 123456\nkernel_sources: {src}\n"
                    f"kernel_sources_sha256: {sha}\n")
    return prof


def test_profiled_traffic_stands_only_for_unchanged_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(_profile(tmp_path, "kernel v1", "kernel v1")))
    assert bench.profiled_traffic("full_frame") == 123456
    assert bench.profiled_traffic("mixed_fp32") is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(_profile(tmp_path, "kernel v2", "kernel v1")))
    assert bench.profiled_traffic("full_frame") is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic("full_frame") is None
