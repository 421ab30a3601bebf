"""Serving with continuous batching: frames of mixed sizes, admitted by HBM
budget, sliced across scheduling steps.  Every result must be bitwise equal to
the same frame run alone; a small frame submitted behind a large one must
finish first; a frame larger than the budget is refused."""
import time

import numpy as np
import pytest

import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_server_results_equal_alone_and_small_frames_overtake():
    import paper_1604_03622_amd as kstap
    plans = {16: kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4), 8: kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3),
             "m": kstap.Plan(p=3, q=16, n=128, r_a=1, r_b=3, precision="bf16x3")}
    frames = [(16, 768, 640), (8, 64, 72), (8, 96, 96), ("m", 200, 180), (16, 90, 70), (8, 300, 260)]
    data = []
    for i, (k, H, W) in enumerate(frames):
        pl = plans[k]
        sc = scenegen.make_scene(scenegen.SceneSpec(p=3, q=pl.q, H=H, W=W, r_b=pl.r_b, n_targets=3), 300 + i)
        data.append((pl, torch.from_numpy(sc.x).pin_memory()))
    print("server: 6 frames", flush=True)
    srv = kstap.Server(hbm_budget_bytes=2 << 30, max_inflight=8, step_pixels=1 << 17)
    tickets = [srv.submit(pl, x) for pl, x in data]
    results = [srv.wait(t, timeout_ms=120000) for t in tickets]
    st = srv.stats()
    print("stats", st, flush=True)
    assert st["frames"] == len(frames) and st["p99_s"] >= st["p50_s"] > 0 and st["pixels_per_s"] > 0
    lat = [r[2] for r in results]
    print("latencies", [f"{v * 1e3:.1f} ms" for v in lat], flush=True)
    # the small q=8 frame submitted right after the large one is done before it
    assert lat[1] < lat[0]
    for (pl, x), (T, D, _) in zip(data, results):
        Ta, Da = kstap.run(pl, x.cuda())
        torch.cuda.synchronize()
        assert torch.equal(T, Ta.cpu()), "served T differs from the frame alone"
        assert torch.equal(D, Da.cpu()), "served D differs from the frame alone"
    # device-resident input
    x = data[1][1].cuda()
    t = srv.submit(plans[8], x)
    T, D, _ = srv.wait(t, timeout_ms=60000)
    assert torch.equal(T, kstap.run(plans[8], x)[0].cpu())
    srv.close()


def test_server_fp32_f64_frames_equal_alone():
    """Frames with FP32 covariance and FP64 solves served beside a plain FP32
    frame: the server's persistent steps give each frame's solo result."""
    import paper_1604_03622_amd as kstap
    plans = [kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4, precision="fp32_f64"),
             kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3, precision="fp32_f64"),
             kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4)]
    data = []
    for i, (pl, H, W) in enumerate(zip(plans, (120, 90, 100), (100, 77, 96))):
        sc = scenegen.make_scene(scenegen.SceneSpec(p=3, q=pl.q, H=H, W=W, r_b=pl.r_b, n_targets=3), 340 + i)
        data.append((pl, torch.from_numpy(sc.x).pin_memory()))
    print("server: 3 frames, two fp32_f64", flush=True)
    srv = kstap.Server(hbm_budget_bytes=1 << 30, max_inflight=4, step_pixels=1 << 13)
    tickets = [srv.submit(pl, x) for pl, x in data]
    results = [srv.wait(t, timeout_ms=120000) for t in tickets]
    for (pl, x), (T, D, _) in zip(data, results):
        Ta, Da = kstap.run(pl, x.cuda())
        torch.cuda.synchronize()
        assert torch.equal(T, Ta.cpu()), f"served T differs from the frame alone ({pl.precision})"
        assert torch.equal(D, Da.cpu()), f"served D differs from the frame alone ({pl.precision})"
    srv.close()


def test_server_budget_admission():
    import paper_1604_03622_amd as kstap
    pl = kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3)
    # a 256 x 256 frame needs 12.3 MiB (input) + 0.3 MiB (outputs): at most three fit in 40 MiB
    srv = kstap.Server(hbm_budget_bytes=40 << 20, max_inflight=16, step_pixels=1 << 16)
    big = torch.zeros((3, 1024, 1024, 8), dtype=torch.complex64)
    with pytest.raises(kstap.StapError) as ei:
        srv.submit(pl, big)
    assert ei.value.status == 5
    xs = [torch.from_numpy(scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=256, W=256, n_targets=1), 400 + i).x)
          .pin_memory() for i in range(6)]
    print("server: 6 frames through a 40 MiB budget", flush=True)
    ts = [srv.submit(pl, x) for x in xs]
    outs = [srv.wait(t, timeout_ms=120000) for t in ts]
    for x, (T, D, _) in zip(xs, outs):
        assert torch.equal(T, kstap.run(pl, x.cuda())[0].cpu())
    srv.close()


def test_server_device_frame_waits_for_its_producer():
    """A device frame still being written on torch's stream when it is
    submitted: the server orders its first read after that work (an event
    recorded on the producer's stream at submit)."""
    import paper_1604_03622_amd as kstap
    pl = kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3)
    sc = scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=200, W=180, n_targets=3), 451)
    src = torch.from_numpy(sc.x).cuda()
    ref, _ = kstap.run(pl, src)
    torch.cuda.synchronize()
    srv = kstap.Server(hbm_budget_bytes=1 << 30, max_inflight=4, step_pixels=1 << 16)
    for trial in range(3):
        print(f"server: device frame written behind a long producer, trial {trial}", flush=True)
        a = torch.randn((4096, 4096), device="cuda")
        y = torch.zeros_like(src)
        for _ in range(4):
            a = a @ a
            a /= a.norm()
        y.copy_(src)   # enqueued behind the products on torch's stream
        t = srv.submit(pl, y)
        T, D, _ = srv.wait(t, timeout_ms=60000)
        assert torch.equal(T, ref.cpu())
    srv.close()
