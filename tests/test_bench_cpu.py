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


def _vectors_by_loop(plan, H, W):
    """Executed vectors recounted position by position: a valid pixel right
    after a valid pixel, inside a sliding-window chain, costs the size of the
    symmetric difference of the two pixels' training sets; others cost n."""
    pix, mv = plan.order(H, W)
    r0, r1, c0, c1 = plan.valid_region(H, W)
    st = {tuple(o) for o in plan.stencil.tolist()}
    total, prev_ok, prev = 0, False, None
    for (r, c), m in zip(pix.tolist(), mv.tolist()):
        ok = r0 <= r < r1 and c0 <= c < c1
        if ok:
            if prev_ok and m >= 0:
                a = {(r + dr, c + dc) for dr, dc in st}
                b = {(prev[0] + dr, prev[1] + dc) for dr, dc in st}
                total += len(a ^ b)
            else:
                total += plan.n
        prev_ok, prev = ok, (r, c)
    return total


@pytest.mark.parametrize("H,W", [(40, 37), (64, 64)])
def test_executed_vectors_match_a_recount(H, W):
    import paper_1604_03622_amd as kstap
    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4)
    vec, npx = bench.executed_vectors(plan, H, W, True)
    assert vec == _vectors_by_loop(plan, H, W)
    r0, r1, c0, c1 = plan.valid_region(H, W)
    assert npx == (r1 - r0) * (c1 - c0)
    assert bench.executed_vectors(plan, H, W, False) == (200.0 * npx, npx)


def test_executed_vectors_on_the_full_frame():
    """2048 x 2048, n = 200: a chain's first pixel sums 200 vectors, the 15
    others 19 + 19: (200 + 15 * 38) / 16 = 48.125 vectors per pixel, up to
    the chains cut by the valid region's edges."""
    import paper_1604_03622_amd as kstap
    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4)
    vec, npx = bench.executed_vectors(plan, 2048, 2048, True)
    assert npx == 2033 * 2033
    assert 48.0 <= vec / npx <= 48.6
    assert bench.slides_for(plan)
    assert not bench.slides_for(kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4, precision="bf16x3"))
    assert bench.slides_for(kstap.Plan(p=5, q=24, n=256, r_a=1, r_b=4, precision="bf16x3"))
