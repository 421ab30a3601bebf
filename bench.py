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
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "full_frame": dict(spec=scenegen.FULL_FRAME, plan=dict(p=3, q=16, n=200, r_a=1, r_b=4, precision="fp32")),
    "tiny": dict(spec=scenegen.TINY, plan=dict(p=3, q=8, n=64, r_a=1, r_b=3, precision="fp32")),
}


def scm_flops_per_pixel(p, q, n):
    """Hermitian sample covariance: 4 n pq (pq + 1) real flops per pixel."""
    pq = p * q
    return 4.0 * n * pq * (pq + 1)


# ----------------------------------------------------------- CPU baseline
_G = {}


def _oracle_chunk(args):
    import oracle
    lo, hi = args
    cfg = oracle.OracleConfig(**_G["ocfg"])
    out = oracle.kron_stap_pixels(_G["x"], _G["pix"][lo:hi], cfg)
    return hi - lo, float(np.nansum(out["T"]))


def cpu_baseline(x, plan_kw, count, seed=123):
    """Times the FP64 oracle (as it stands; not tuned) on `count` seeded valid
    pixels of the same frame, one process per core, BLAS threads = 1."""
    import oracle
    os.environ["OMP_NUM_THREADS"] = "1"
    ocfg = dict(p=plan_kw["p"], q=plan_kw["q"], n=plan_kw["n"], r_a=plan_kw["r_a"], r_b=plan_kw["r_b"])
    H, W = x.shape[1], x.shape[2]
    region = oracle.valid_region(H, W, oracle.OracleConfig(**ocfg).training_stencil())
    pix = scenegen.random_pixels(H, W, count, seed, region=region)
    _G.update(x=x, pix=pix, ocfg=ocfg)
    cores = min(16, len(os.sched_getaffinity(0)))
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
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return dict(value=done / dt, unit="pixels/s", cores=cores, kind="oracle",
                sample=f"{done} seeded valid pixels of the same frame, FP64 NumPy, {dt:.1f} s wall")


# ------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="full_frame", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=400000)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(pixels are independent given their halo; see DESIGN.md for the multi-GPU layout)",
              file=sys.stderr)
        sys.exit(2)

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

    flops = scm_flops_per_pixel(plan_kw["p"], plan_kw["q"], plan_kw["n"]) * valid_px
    achieved = flops / (ms_per_step / 1e3) / 1e12
    result = {
        "metric": "Kron-STAP output pixels/s on 1 MI355X (plain FP32 path)",
        "value": px_s,
        "unit": "pixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
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
            "peak": MFMA_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / MFMA_FP32_PEAK_TFLOPS,
            "traffic": None,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
