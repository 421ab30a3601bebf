"""Benchmark: Kron-STAP output pixels/s on one MI355X.

Workload (default): one full synthetic frame, p=3 channels, q=16 azimuth
samples, 2048 x 2048 pixels complex64, n=200 training snapshots per pixel
(16 x 16 window minus a 3 x 3 guard), rank(A)=1, rank(B)=4, factors rotating
per 256-pixel block, 200 targets; plain FP32 path.  A "step" is one whole
frame pass (covariance, LR-Kron, subspaces, statistic, detection) with the
frame already resident in HBM.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build measures one GPU.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import scenegen  # noqa: E402

MFMA_FP32_PEAK_TFLOPS = 157.3
MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "full_frame": dict(spec=scenegen.FULL_FRAME, plan=dict(p=3, q=16, n=200, r_a=1, r_b=4, precision="fp32")),
    "tiny": dict(spec=scenegen.TINY, plan=dict(p=3, q=8, n=64, r_a=1, r_b=3, precision="fp32")),
    # for profiling the other kernels under the same harness
    "full_frame_bf16x3": dict(spec=scenegen.FULL_FRAME, plan=dict(p=3, q=16, n=200, r_a=1, r_b=4, precision="bf16x3")),
    "mixed_fp32": dict(spec=scenegen.MIXED, plan=dict(p=5, q=24, n=256, r_a=1, r_b=4, precision="fp32")),
    "mixed_bf16x3": dict(spec=scenegen.MIXED, plan=dict(p=5, q=24, n=256, r_a=1, r_b=4, precision="bf16x3")),
}


# rocprofv3 summary of the dominant kernel on the full frame: its HBM bytes
# per launch (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size) stand
# only while the kernel sources hash to the value recorded beside them.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "kstap_kernel_p3q16_full_frame_fp32.md")


def profiled_traffic(workload):
    if workload != "full_frame" or not os.path.exists(TRAFFIC_PROFILE):
        return None
    import hashlib
    fields = {}
    for line in open(TRAFFIC_PROFILE):
        k, sep, v = line.partition(":")
        if sep and k in ("traffic_bytes_per_launch", "kernel_sources", "kernel_sources_sha256"):
            fields[k] = v.strip()
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for f in fields["kernel_sources"].split():
        path = os.path.join(ROOT, f)
        if not os.path.exists(path):
            return None
        with open(path, "rb") as fh:
            h.update(fh.read())
    return int(fields["traffic_bytes_per_launch"]) if h.hexdigest() == fields["kernel_sources_sha256"] else None


def scm_flops_per_pixel(p, q, n):
    """Hermitian sample covariance: 4 n pq (pq + 1) real flops per pixel."""
    pq = p * q
    return 4.0 * n * pq * (pq + 1)


def executed_vectors(plan, H, W, slides):
    """Training vectors the frame pass accumulates into covariances, summed
    over the frame's valid pixels, from the plan's visiting order and its
    sliding-window lists: a pixel whose position continues a chain and whose
    predecessor in the order is a valid pixel updates that pixel's n S with
    the vectors entering and leaving the stencil; every other valid pixel sums
    all n.  `slides` is False for kernels that always take the full sum (the
    narrow kernels with FP64 solves).  Returns (vectors, valid pixels)."""
    pix, mv = plan.order(H, W)
    r0, r1, c0, c1 = plan.valid_region(H, W)
    valid = (pix[:, 0] >= r0) & (pix[:, 0] < r1) & (pix[:, 1] >= c0) & (pix[:, 1] < c1)
    npx = int(valid.sum())
    if not slides or plan.moves(0) is None:
        return float(plan.n) * npx, npx
    prev = np.concatenate([[False], valid[:-1]])
    slide = valid & prev & (mv >= 0)
    delta = np.zeros(3)
    for m in range(3):
        add, rem = plan.moves(m)
        delta[m] = len(add) + len(rem)
    vec = float(plan.n) * int((valid & ~slide).sum()) + float(delta[mv[slide]].sum())
    return vec, npx


def slides_for(plan):
    """Whether the plan's kernel updates covariances along sliding-window
    chains (FP32 narrow kernels and both wide kernels)."""
    return plan.precision == "fp32" or plan.p * plan.q > 64


# ----------------------------------------------------------- CPU baseline
_G = {}


def _oracle_chunk(args):
    import oracle
    lo, hi = args
    cfg = oracle.OracleConfig(**_G["ocfg"])
    out = oracle.kron_stap_pixels(_G["x"], _G["pix"][lo:hi], cfg)
    return hi - lo, float(np.nansum(out["T"]))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


# Worker processes of the CPU leg: the host cores given to one GPU (16 on the
# measurement hosts), or fewer if fewer are available to this process.
CPU_SHARE = 16


def cpu_baseline(x, plan_kw, count, seed=123, single=20000):
    """Times the FP64 oracle (as it stands; not tuned) on `count` seeded valid
    pixels of the same frame, one process per core of the host share, BLAS
    threads = 1; then `single` of those pixels in one process (the
    single-core rate)."""
    import oracle
    os.environ["OMP_NUM_THREADS"] = "1"
    ocfg = dict(p=plan_kw["p"], q=plan_kw["q"], n=plan_kw["n"], r_a=plan_kw["r_a"], r_b=plan_kw["r_b"])
    H, W = x.shape[1], x.shape[2]
    region = oracle.valid_region(H, W, oracle.OracleConfig(**ocfg).training_stencil())
    pix = scenegen.random_pixels(H, W, count, seed, region=region)
    _G.update(x=x, pix=pix, ocfg=ocfg)
    cores = min(CPU_SHARE, len(os.sched_getaffinity(0)))
    step = max(1, count // (cores * 4))
    chunks = [(lo, min(count, lo + step)) for lo in range(0, count, step)]
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover - threadpoolctl is optional
        limiter = None
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        done = sum(n for n, _ in pool.map(_oracle_chunk, chunks))
    dt = time.perf_counter() - t0
    single = min(single, count)
    t1 = time.perf_counter()
    _oracle_chunk((0, single))
    dt1 = time.perf_counter() - t1
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return dict(value=done / dt, unit="pixels/s", cores=cores, kind="oracle",
                sample=f"{done} seeded valid pixels of the same frame, FP64 NumPy, {dt:.1f} s wall on {cores} "
                       f"processes; single core: {single} of them in {dt1:.1f} s",
                single_core_value=single / dt1, cpu_model=cpu_model(),
                host_cores_visible=len(os.sched_getaffinity(0)))


# ------------------------------------------------------------ system forms
def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _roofs(plan, H, W, sec, prec):
    """Covariance work the kernel executes per second against the MFMA roof
    of the arithmetic it runs on: FP32 MFMA for the plain path; for the
    split-BF16 path the BF16 peak divided by its three products (the bf16x3
    roof) and the BF16 peak itself (the stricter roof of a single product)."""
    pq = plan.p * plan.q
    vec, npx = executed_vectors(plan, H, W, slides_for(plan))
    tfl = vec * 4.0 * pq * (pq + 1) / sec / 1e12
    out = dict(vectors_per_pixel=vec / npx, executed_scm_tflops=tfl,
               dense_equivalent_tflops=scm_flops_per_pixel(plan.p, plan.q, plan.n) * npx / sec / 1e12)
    if prec == "bf16x3":
        out.update(frac_bf16x3_roof=tfl / (MFMA_BF16_PEAK_TFLOPS / 3.0), frac_bf16_k1_roof=tfl / MFMA_BF16_PEAK_TFLOPS)
    else:
        out.update(frac_fp32_mfma_roof=tfl / MFMA_FP32_PEAK_TFLOPS)
    return out


def form_frame_mixed(kstap, torch, scene, steps, prec="bf16x3"):
    """The same full frame with split-BF16 covariance and FP64 eigensolves
    (bf16x3), or FP32 covariance full sums and FP64 eigensolves (fp32_f64)."""
    x = torch.from_numpy(scene.x).cuda()
    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4, precision=prec)
    H, W = x.shape[1], x.shape[2]
    T = torch.empty(x.shape[1:3], device="cuda")
    D = torch.empty(x.shape[1:3], dtype=torch.uint8, device="cuda")
    r0, r1, c0, c1 = plan.valid_region(H, W)
    sec = _timed(torch, lambda: kstap.run(plan, x, T, D), steps)
    px = (r1 - r0) * (c1 - c0)
    cov = "bf16x3 covariance" if prec == "bf16x3" else "FP32 covariance (full sums)"
    out = dict(workload=f"full frame 2048x2048 p=3 q=16 n=200, {cov} + FP64 eigensolves",
               pixels_per_s=px / sec, ms=sec * 1e3,
               bound="valu (FP64 solves; see the kernel profile)")
    out.update(_roofs(plan, H, W, sec, prec))
    return out


def form_wide_mixed(kstap, torch, steps):
    """Mixed-precision workload: p=5, q=24 (pq=120), 1024 x 1024, n=256, split-BF16
    covariance with FP64 eigensolves, against the plain FP32 path on the same frame."""
    sc = scenegen.make_scene(scenegen.MIXED)
    x = torch.from_numpy(sc.x).cuda()
    del sc
    H, W = x.shape[1], x.shape[2]
    out = dict(workload="p=5 q=24 1024x1024 complex64, n=256, r_a=1 r_b=4")
    for prec in ("fp32", "bf16x3"):
        plan = kstap.Plan(p=5, q=24, n=256, r_a=1, r_b=4, precision=prec)
        T = torch.empty(x.shape[1:3], device="cuda")
        D = torch.empty(x.shape[1:3], dtype=torch.uint8, device="cuda")
        r0, r1, c0, c1 = plan.valid_region(H, W)
        px = (r1 - r0) * (c1 - c0)
        sec = _timed(torch, lambda: kstap.run(plan, x, T, D), steps)
        out[prec] = dict(pixels_per_s=px / sec, ms=sec * 1e3)
        out[prec].update(_roofs(plan, H, W, sec, prec))
        _log(f"wide {prec}: {px / sec / 1e6:.2f} Mpx/s")
    return out


def form_batch(kstap, torch):
    """64 uneven tiles: per-tile plain FP32 path vs one batched launch (FP32
    and split-BF16)."""
    specs = scenegen.batch_tile_specs()
    xs, outs = [], []
    for i, (sp, n) in enumerate(specs):
        xs.append(scenegen.make_scene_torch(sp, seed=scenegen.BASE_SEED + 100 + i))
        outs.append((torch.empty((sp.H, sp.W), device="cuda"), torch.empty((sp.H, sp.W), dtype=torch.uint8, device="cuda")))
    torch.cuda.synchronize()
    px = sum(sp.H * sp.W for sp, _ in specs)
    res = dict(workload=f"{len(specs)} tiles, side in {{128..1024}}, q in {{8,12,16}}, n in {{64,128,256}}, "
                        f"r_a in {{1,2}}, r_b in {{2..6}}", pixels=px)
    for prec in ("fp32", "bf16x3"):
        plans = [kstap.Plan(p=3, q=sp.q, n=n, r_a=sp.r_a, r_b=sp.r_b, precision=prec) for sp, n in specs]
        tiles = [(pl, x, T, D) for pl, x, (T, D) in zip(plans, xs, outs)]
        if prec == "fp32":
            sec = _timed(torch, lambda: [kstap.run(pl, x, T, D) for pl, x, T, D in tiles], 2)
            res["per_tile_fp32_pixels_per_s"] = px / sec
        b = kstap.Batch(tiles)
        tuned = b.tune()
        sec = _timed(torch, b.launch, 3)
        res[f"batched_{prec}_pixels_per_s"] = px / sec
        res[f"batched_{prec}_tuned"] = tuned
        _log(f"batch {prec}: {px / sec / 1e6:.1f} Mpx/s")
    return res


def form_serving(kstap, torch, nframes, pool=40):
    """Poisson stream (and a burst) of frames of mixed sizes through the
    continuous-batching server vs the plain per-frame path (upload, run,
    download, one frame at a time), same arrival trace, latency = submit to
    results in host memory.  The `nframes` arrivals draw from a pool of
    `pool` distinct seeded frames (pinned host memory holds the pool, not
    every arrival)."""
    import threading
    trace = scenegen.serving_trace()[:pool]
    pooled = []
    for i, (sp, n) in enumerate(trace):
        xd = scenegen.make_scene_torch(sp, seed=scenegen.BASE_SEED + 500 + i)
        xh = torch.empty(xd.shape, dtype=torch.complex64, pin_memory=True)
        xh.copy_(xd)
        del xd
        pooled.append((kstap.Plan(p=3, q=sp.q, n=n, r_a=1, r_b=3), xh, sp.H * sp.W,
                       kstap.Plan(p=3, q=sp.q, n=n, r_a=1, r_b=3, precision="bf16x3")))
    pick = np.random.Generator(np.random.PCG64(scenegen.BASE_SEED + 8)).integers(0, len(pooled), nframes)
    frames = [pooled[k] for k in pick]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    tot_px = sum(f[2] for f in frames)
    mean_px = tot_px / len(frames)

    def plain(arrivals):
        lat = []
        t0 = time.perf_counter()
        for (pl, xh, npx, _), ta in zip(frames, arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            xd = xh.to("cuda", non_blocking=True)
            T, D = kstap.run(pl, xd)
            Th, Dh = T.cpu(), D.cpu()
            lat.append(time.perf_counter() - t0 - ta)
            del xd
        span = time.perf_counter() - t0
        return lat, span

    def served(arrivals, mixed=False):
        srv = kstap.Server(hbm_budget_bytes=24 << 30, max_inflight=16, step_pixels=1 << 20)
        tickets = []
        t0 = time.perf_counter()

        def submit():
            for (pl, xh, npx, plm), ta in zip(frames, arrivals):
                now = time.perf_counter() - t0
                if ta > now:
                    time.sleep(ta - now)
                tickets.append(srv.submit(plm if mixed else pl, xh))
        th = threading.Thread(target=submit)
        th.start()
        th.join()
        lat = [srv.wait(t)[2] for t in tickets]
        span = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return lat, span, st

    # capacity of the plain path on this trace (all frames queued at once)
    lat0, span0 = plain([0.0] * len(frames))
    cap_fps = len(frames) / span0
    rate = 0.7 * cap_fps
    rng = np.random.Generator(np.random.PCG64(scenegen.BASE_SEED + 9))
    arr = np.cumsum(rng.exponential(1.0 / rate, len(frames)))
    arr -= arr[0]
    out = dict(workload=f"{len(frames)} arrivals drawn from {len(pooled)} distinct frames, side U{{256..2048}}, "
                        f"q in {{8,16}}, n U{{64..256}}, p=3; pinned host frames, latency = submit to results in "
                        f"host memory",
               frames=len(frames), distinct_frames=len(pooled), mean_pixels_per_frame=mean_px,
               poisson_rate_fps=rate, rate_rule="0.7 x plain-path capacity on this trace")
    for name, arrivals in (("burst", [0.0] * len(frames)), ("poisson", list(arr))):
        pl_lat, pl_span = plain(arrivals)
        sv_lat, sv_span, st = served(arrivals)
        mx_lat, mx_span, mst = served(arrivals, mixed=True)
        out[name] = dict(
            plain=dict(pixels_per_s=tot_px / pl_span, p50_s=float(np.percentile(pl_lat, 50)),
                       p99_s=float(np.percentile(pl_lat, 99))),
            server=dict(pixels_per_s=tot_px / sv_span, p50_s=float(np.percentile(sv_lat, 50)),
                        p99_s=float(np.percentile(sv_lat, 99)), server_stats=st),
            server_bf16x3=dict(pixels_per_s=tot_px / mx_span, p50_s=float(np.percentile(mx_lat, 50)),
                               p99_s=float(np.percentile(mx_lat, 99)), server_stats=mst),
            mixed_served_over_plain_fp32=pl_span / mx_span)
        _log(f"serving {name}: server {tot_px / sv_span / 1e6:.1f} Mpx/s p99 {np.percentile(sv_lat, 99) * 1e3:.0f} ms; "
             f"server bf16x3 {tot_px / mx_span / 1e6:.1f} Mpx/s p99 {np.percentile(mx_lat, 99) * 1e3:.0f} ms; "
             f"plain {tot_px / pl_span / 1e6:.1f} Mpx/s p99 {np.percentile(pl_lat, 99) * 1e3:.0f} ms")
    return out


def measured_peaks(torch):
    """Throughput measured on this GPU with plain library operations, as lower
    bounds of its peaks: HBM bandwidth of a 1 GiB device-to-device copy
    (bytes read + written over time) and torch.matmul at 8192^3 in FP32 and
    BF16 (dense GEMM on the matrix cores)."""
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sec = _timed(torch, lambda: dst.copy_(src), 10)
    out = dict(hbm_copy_GBps=2 * (1 << 30) / sec / 1e9)
    del src, dst
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
        a = torch.randn((8192, 8192), device="cuda").to(dt)
        b = torch.randn((8192, 8192), device="cuda").to(dt)
        sec = _timed(torch, lambda: torch.matmul(a, b), 5)
        out[f"{name}_gemm_TFLOPs"] = 2 * 8192 ** 3 / sec / 1e12
        del a, b
    torch.cuda.empty_cache()
    out["note"] = "lower bounds of the hardware peaks; roofline fractions use the published peaks"
    return out


def form_large_q(kstap, torch, cpu=True):
    """LR-Kron on one large covariance, the paper's timing workload: n = 5
    snapshots, a rank-one space factor, identity time factor, p = 3 with q up
    to 2500 and p = 6 with q up to 1250, tolerances 1e-4 and 1e-6.  Time per
    estimate (A-hat, eta and the q x q B-hat), the solve alone, and the FP64
    oracle on the same snapshots."""
    import oracle.large_q as LQ
    rows = []
    for p, qs in ((3, (50, 250, 500, 1000, 2500)), (6, (25, 250, 1250))):
        for q in qs:
            X = scenegen.large_q_snapshots(p, q, 5, seed=scenegen.BASE_SEED + 1000 + q)
            xd = torch.from_numpy(X).cuda()
            for eps in (1e-4, 1e-6):
                out = kstap.lrkron(xd, eps=eps)
                torch.cuda.synchronize()
                st = out["stats"].cpu().numpy()
                full = _timed(torch, lambda: kstap.lrkron(xd, eps=eps), 20)
                solve = _timed(torch, lambda: kstap.lrkron(xd, eps=eps, with_B=False), 20)
                row = dict(p=p, q=q, n=5, eps=eps, iterations=int(st[1]), eta=float(st[0]), us_total=full * 1e6,
                           us_solve=solve * 1e6,
                           emit_b_GBps=q * q * 8 / max(full - solve, 1e-9) / 1e9)
                if cpu and q <= 1000:
                    t0 = time.perf_counter()
                    LQ.lr_kron_snapshots(X, eps=eps)
                    row["oracle_s"] = time.perf_counter() - t0
                rows.append(row)
                _log(f"large q p={p} q={q} eps={eps:g}: {full * 1e6:.1f} us ({int(st[1])} iterations)")
    return dict(workload="one covariance from n=5 snapshots, rank-one A, B = I_q (Sec. 6.1 timing setting)",
                rows=rows,
                note="B-hat emission is bound by writing q^2 complex64 values; emit_b_GBps = q^2 * 8 bytes over "
                     "(total - solve) time")


def form_variants(kstap, torch):
    """Statistic variants on a 1024 x 1024 p=3 q=16 frame (FP32): the plain
    statistic, the classical projector, a 16-bin Doppler bank with the
    enhancement image and bin map, and a two-pass 512 x 512 multipass frame
    with its per-pass and change images."""
    spec = scenegen.SceneSpec(p=3, q=16, H=1024, W=1024, r_a=1, r_b=4, n_targets=50, snr_db=(0.0, 15.0), block=256)
    x = scenegen.make_scene_torch(spec, seed=scenegen.BASE_SEED + 1200)
    base = dict(p=3, q=16, n=200, r_a=1, r_b=4)
    plans = dict(plain=kstap.Plan(**base), classical=kstap.Plan(**base, filter="classical"),
                 bank16_enhancement=kstap.Plan(**base, nbank=16))
    H, W = spec.H, spec.W
    r0, r1, c0, c1 = plans["plain"].valid_region(H, W)
    px = (r1 - r0) * (c1 - c0)
    out = dict(workload="1024x1024 p=3 q=16 n=200 FP32; multipass 2 x 3 channels 512x512 q=16 n=200")
    for name, pl in plans.items():
        sec = _timed(torch, lambda: kstap.run_ex(pl, x), 3)
        out[name] = dict(pixels_per_s=px / sec, ms=sec * 1e3)
        _log(f"variant {name}: {px / sec / 1e6:.1f} Mpx/s")
    del x
    mp = scenegen.make_multipass_scene(scenegen.MultipassSpec(passes=2, p=3, q=16, H=512, W=512, r_b=4, n_targets=20),
                                       seed=scenegen.BASE_SEED + 1201)
    xm = torch.from_numpy(mp.x).cuda()
    pl = kstap.Plan(p=6, q=16, n=200, r_a=2, r_b=4, passes=2)
    r0, r1, c0, c1 = pl.valid_region(512, 512)
    sec = _timed(torch, lambda: kstap.run_ex(pl, xm), 3)
    out["multipass_k2"] = dict(pixels_per_s=(r1 - r0) * (c1 - c0) / sec, ms=sec * 1e3)
    _log(f"variant multipass: {(r1 - r0) * (c1 - c0) / sec / 1e6:.2f} Mpx/s")
    return out


def form_robustness(kstap, torch, cpu=True):
    """Robustness evaluation (Sec. 2 SIRV model, Sec. 5 filters): a 256 x 256
    p=3 q=16 scene with K-distributed texture (nu = 0.5) and, around each of
    64 test pixels, 6 movers at 25 dB inside the training window, all with
    the steering a(1.2) (x) b(0.2).  Times the LR-STAP baseline on every valid
    pixel and the SINR-loss kernel on the test pixels over 2 x 65 steerings,
    and reports the mean SINR loss of Kron-STAP, the classical joint
    projector and LR-STAP (rank r_a r_b and r_a r_b + 1) at the movers'
    steering and over the Doppler grid."""
    spec = scenegen.SirvSpec(p=3, q=16, H=256, W=256, r_b=4, texture_nu=0.5, n_test=64, margin=16, n_corrupt=6,
                             radius=7, corrupt_snr_db=25.0, corrupt_theta=1.2, corrupt_f=0.2)
    sc = scenegen.make_sirv_scene(spec, seed=scenegen.BASE_SEED + 1300)
    n, ra, rb = 200, 1, 4
    plan = kstap.Plan(p=3, q=16, n=n, r_a=ra, r_b=rb)
    x = torch.from_numpy(sc.x).cuda()
    r0, r1, c0, c1 = plan.valid_region(spec.H, spec.W)
    rr, cc = np.meshgrid(np.arange(r0, r1), np.arange(c0, c1), indexing="ij")
    allpix = np.stack([rr.ravel(), cc.ravel()], 1).astype(np.int32)
    pix_t = torch.from_numpy(allpix).cuda()
    sec_lr = _timed(torch, lambda: kstap.lrstap_probe(plan, x, pix_t, r=ra * rb), 3)
    pq = 3 * 16
    scm_flops = 8.0 * n * pq * (pq + 1) / 2                     # FP32 S accumulation, upper triangle
    out = dict(workload="SIRV 256x256 p=3 q=16 n=200, K-distributed texture nu=0.5, 6 movers (25 dB) in the "
                        "training window of each of 64 test pixels",
               lrstap=dict(pixels=int(len(allpix)), pixels_per_s=len(allpix) / sec_lr, ms=sec_lr * 1e3,
                           scm_tflops=len(allpix) * scm_flops / sec_lr / 1e12,
                           note="one 64-lane workgroup per pixel; S by VALU (FP32), subspace iteration FP64"))
    _log(f"robustness: LR-STAP {len(allpix) / sec_lr / 1e6:.2f} Mpx/s")
    tp = sc.test_pixels
    pr = kstap.probe(plan, x, tp)
    lr = {r: kstap.lrstap_probe(plan, x, tp, r=r) for r in (ra * rb, ra * rb + 1)}
    fgrid = np.linspace(-0.5, 0.5, 65)
    a_grid = np.stack([scenegen.spatial_steering(3, t) for t in (1.2, 2.5)]).astype(np.complex64)
    b_grid = np.stack([scenegen.doppler_steering(16, f) for f in fgrid]).astype(np.complex64)
    tc = (sc.UA.astype(np.complex64), sc.lamA, sc.UB.astype(np.complex64), sc.lamB, sc.sigma2, sc.tau2_mean)
    losses = {k: kstap.sinr_loss(k, a_grid, b_grid, *tc, UA=pr["U_A"], UB=pr["U_B"]) for k in ("kron", "classical")}
    for r, o in lr.items():
        losses[f"lrstap_r{r}"] = kstap.sinr_loss("lrstap", a_grid, b_grid, *tc, U=o["U"])
    sec_s = _timed(torch, lambda: kstap.sinr_loss("kron", a_grid, b_grid, *tc, UA=pr["U_A"], UB=pr["U_B"]), 5)
    fi = int(np.argmin(np.abs(fgrid - 0.2)))
    db = lambda v: float(10.0 * np.log10(max(float(v), 1e-30)))  # noqa: E731
    curves = {}
    for k, L in losses.items():
        Lc = L.cpu().numpy()
        curves[k] = dict(at_movers_db=db(Lc[:, 0, fi].mean()), mean_db_theta1p2=db(Lc[:, 0, :].mean()),
                         mean_db_theta2p5=db(Lc[:, 1, :].mean()),
                         curve_db_theta1p2=[round(db(v), 3) for v in Lc[:, 0, :].mean(axis=0)])
    out["sinr"] = dict(test_pixels=int(len(tp)), steerings=int(a_grid.shape[0] * b_grid.shape[0]),
                       evaluations_per_s=len(tp) * a_grid.shape[0] * b_grid.shape[0] / sec_s, ms=sec_s * 1e3,
                       doppler_grid=[float(f) for f in fgrid], curves=curves)
    _log("robustness: loss at the movers' steering (dB): " +
         ", ".join(f"{k} {v['at_movers_db']:.1f}" for k, v in curves.items()))
    if cpu:
        import oracle
        import oracle.robustness as RB
        cfg = oracle.OracleConfig(p=3, q=16, n=n, r_a=ra, r_b=rb)
        t0 = time.perf_counter()
        RB.lr_stap_pixels(sc.x, allpix[:2000], cfg, r=ra * rb)
        out["lrstap"]["oracle_pixels_per_s_one_process"] = 2000 / (time.perf_counter() - t0)
    return out


def system_forms(kstap, torch, args, scene):
    forms = {}
    forms["frame_bf16x3"] = form_frame_mixed(kstap, torch, scene, max(3, args.steps // 2))
    _log(f"frame bf16x3: {forms['frame_bf16x3']['pixels_per_s'] / 1e6:.1f} Mpx/s")
    forms["frame_fp32_f64"] = form_frame_mixed(kstap, torch, scene, max(3, args.steps // 2), "fp32_f64")
    _log(f"frame fp32_f64: {forms['frame_fp32_f64']['pixels_per_s'] / 1e6:.1f} Mpx/s")
    torch.cuda.empty_cache()
    forms["mixed_workload"] = form_wide_mixed(kstap, torch, 3)
    torch.cuda.empty_cache()
    forms["batch"] = form_batch(kstap, torch)
    torch.cuda.empty_cache()
    forms["serving"] = form_serving(kstap, torch, args.serve_frames)
    torch.cuda.empty_cache()
    forms["large_q"] = form_large_q(kstap, torch, cpu=not args.no_cpu)
    torch.cuda.empty_cache()
    forms["variants"] = form_variants(kstap, torch)
    torch.cuda.empty_cache()
    forms["robustness"] = form_robustness(kstap, torch, cpu=not args.no_cpu)
    return forms


# ------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="full_frame", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=400000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched / served / mixed-precision legs")
    ap.add_argument("--serve-frames", type=int, default=300)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--only-form", choices=("large_q", "variants", "robustness", "frame_precisions"),
                    help="run one secondary form alone and print its JSON (for kernel profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(pixels are independent given their halo: a frame would shard into row bands, "
              "one per GPU, each with the stencil's halo rows)",
              file=sys.stderr)
        sys.exit(2)

    if args.only_form:
        import torch
        import paper_1604_03622_amd as kstap
        if args.only_form == "large_q":
            out = form_large_q(kstap, torch, cpu=False)
        elif args.only_form == "robustness":
            out = form_robustness(kstap, torch, cpu=False)
        elif args.only_form == "frame_precisions":
            scene = scenegen.make_scene(WORKLOADS["full_frame"]["spec"])
            out = {prec: form_frame_mixed(kstap, torch, scene, max(3, args.steps // 2), prec)
                   for prec in ("bf16x3", "fp32_f64")}
        else:
            out = form_variants(kstap, torch)
        if args.calibrate_copy:
            src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
            dst = src.clone()
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps({"form": args.only_form, "result": out}), flush=True)
        return

    wl = WORKLOADS[args.workload]
    spec, plan_kw = wl["spec"], wl["plan"]
    t0 = time.perf_counter()
    scene = scenegen.make_scene(spec)
    print(f"[bench] scene {spec.p}x{spec.H}x{spec.W}x{spec.q} generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(scene.x, plan_kw, args.cpu_sample)
        print(f"[bench] cpu baseline {cpu['value']:.1f} px/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch
    import paper_1604_03622_amd as kstap

    dev = torch.device("cuda:0")
    x = torch.from_numpy(scene.x).to(dev)
    plan = kstap.Plan(**plan_kw)
    H, W = spec.H, spec.W
    r0, r1, c0, c1 = plan.valid_region(H, W)
    valid_px = (r1 - r0) * (c1 - c0)
    T = torch.empty((H, W), dtype=torch.float32, device=dev)
    D = torch.empty((H, W), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        kstap.run(plan, x, T, D, stream=stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        kstap.run(plan, x, T, D, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    px_s = valid_px * args.steps / (ms_total / 1e3)
    det = int(D.sum().item())

    # roofline of the frame kernel: the covariance is the dense contraction
    # (MFMA); credited with the work the kernel executes (vectors actually
    # accumulated, sliding-window updates included), 4 pq (pq+1) flops per
    # vector and pixel
    mixed = plan_kw["precision"] == "bf16x3"
    pq = plan_kw["p"] * plan_kw["q"]
    vec, npx = executed_vectors(plan, H, W, slides_for(plan))
    assert npx == valid_px
    flops = vec * 4.0 * pq * (pq + 1)
    achieved = flops / (ms_per_step / 1e3) / 1e12
    dense = scm_flops_per_pixel(plan_kw["p"], plan_kw["q"], plan_kw["n"]) * valid_px / (ms_per_step / 1e3) / 1e12
    # the split-BF16 path runs three BF16 products per FP32-class product
    peak = MFMA_BF16_PEAK_TFLOPS / 3 if mixed else MFMA_FP32_PEAK_TFLOPS
    result = {
        "metric": "Kron-STAP output pixels/s on 1 MI355X (" +
                  ("split-BF16 covariance, FP64 solves" if mixed else "plain FP32 path") + ")",
        "value": px_s,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3+f64" if mixed else "f32",
        "data": "synthetic Kronecker-clutter scene (seeded), resident in HBM",
        "config": {
            "workload": f"{args.workload}: p={plan_kw['p']} q={plan_kw['q']} {H}x{W} complex64, n={plan_kw['n']}, "
                        f"r_a={plan_kw['r_a']} r_b={plan_kw['r_b']}, {plan_kw['precision']}",
            "valid_pixels": valid_px,
            "detections": det,
            "wall_s": wall,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": profiled_traffic(args.workload),   # HBM bytes per launch, rocprofv3 counters
            "credited": f"executed covariance work: {vec / valid_px:.3f} training vectors per valid pixel "
                        f"(sliding-window updates counted as the vectors they add and remove) x 4 pq (pq+1) "
                        f"flops; one launch = {valid_px} valid pixels",
            "vectors_per_pixel": vec / valid_px,
            "flops_per_launch": flops,
            "dense_equivalent_tflops": dense,
            "dense_equivalent_note": "4 n pq (pq+1) flops per valid pixel, the direct definition of the "
                                     "covariance; not executed by the sliding-window kernel",
        },
        "cpu_baseline": cpu,
    }
    if not args.no_forms:
        del x
        torch.cuda.empty_cache()
        result["measured_peaks"] = measured_peaks(torch)
        result["forms"] = system_forms(kstap, torch, args, scene)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
