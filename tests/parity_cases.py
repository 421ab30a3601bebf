"""Scenes and configurations of the GPU parity tests (no GPU needed here).

Each case is (scene spec, seed, plan/oracle keywords, precision).  The GPU
tests run the HIP path on the case's scene and compare it with the FP64
oracle; `tests/test_parity_cases_cpu.py` checks on the CPU, with the oracle
alone, that every case grades most of its valid pixels (so that no GPU parity
test can pass on an empty or tiny graded set) and that the cases reach every
kernel class the library builds.
"""
import numpy as np

import scenegen

# ---------------------------------------------------------- configuration variants
VARIANTS = ["n61", "n256", "custom_stencil", "fixed_h", "rb0", "bsteer", "ra2_p4", "q12_rb6", "p2_q32",
            "eps0_iters3"]


def variant_case(case):
    base = dict(p=3, q=8, n=64, r_a=1, r_b=3)
    spec = dict(p=3, q=8, H=40, W=44, r_a=1, r_b=3, n_targets=4)
    if case == "n61":
        base.update(n=61)
    elif case == "n256":
        base.update(n=256)
        spec.update(H=44, W=44)
    elif case == "custom_stencil":
        rng = np.random.default_rng(3)
        cand = [(a, b) for a in range(-6, 7) for b in range(-6, 7) if (a, b) != (0, 0)]
        sel = rng.permutation(len(cand))[:50]
        base.update(n=50, stencil=np.array([cand[i] for i in sel]))
    elif case == "fixed_h":
        base.update(stat_mode="fixed", h_steer=np.exp(1j * 0.8 * np.arange(3)))
    elif case == "rb0":
        base.update(r_b=0)
    elif case == "bsteer":
        bs = np.exp(1j * 0.3 * np.arange(8))
        base.update(b_steer=bs)
        spec.update(b_steer=tuple(bs))
    elif case == "ra2_p4":
        base.update(p=4, r_a=2)
        spec.update(p=4, r_a=2)
    elif case == "q12_rb6":
        base.update(q=12, r_b=6, n=128)
        spec.update(q=12, r_b=6)
    elif case == "p2_q32":
        base.update(p=2, q=32, r_b=4, n=128)
        spec.update(p=2, q=32, r_b=4)
    elif case == "eps0_iters3":
        base.update(eps=0.0, max_iter=3)
    else:
        raise KeyError(case)
    return scenegen.SceneSpec(**spec), 100 + len(case), base, "fp32"


# ------------------------------------------------------------ mixed precision
MIXED = ["tiny", "frame_q16", "q12_rb6", "q8_rb8_ra2", "fixed_h"]


def mixed_case(case):
    if case == "tiny":
        spec = scenegen.TINY
        base = dict(p=3, q=8, n=64, r_a=1, r_b=3)
    elif case == "frame_q16":
        spec = scenegen.SceneSpec(p=3, q=16, H=72, W=72, r_a=1, r_b=4, n_targets=6, snr_db=(0.0, 15.0), block=24)
        base = dict(p=3, q=16, n=200, r_a=1, r_b=4)
    elif case == "q12_rb6":
        spec = scenegen.SceneSpec(p=3, q=12, H=44, W=40, r_a=1, r_b=6, n_targets=4)
        base = dict(p=3, q=12, n=128, r_a=1, r_b=6)
    elif case == "q8_rb8_ra2":
        spec = scenegen.SceneSpec(p=3, q=8, H=40, W=40, r_a=2, r_b=5, n_targets=4)
        base = dict(p=3, q=8, n=64, r_a=2, r_b=5)
    elif case == "fixed_h":
        spec = scenegen.SceneSpec(p=3, q=16, H=40, W=40, r_a=1, r_b=4, n_targets=4)
        base = dict(p=3, q=16, n=200, r_a=1, r_b=4, stat_mode="fixed", h_steer=np.exp(0.6j * np.arange(3)))
    else:
        raise KeyError(case)
    return spec, scenegen.BASE_SEED + 50 + len(case), base, "bf16x3"


# ---------------------------------------------------------------- wide pixels
WIDE = ["p5q24_fp32", "p5q24_bf16x3", "p6q16_ra2_fp32", "p6q16_ra2_bf16x3"]


def wide_case(case):
    prec = "bf16x3" if case.endswith("bf16x3") else "fp32"
    if case.startswith("p5"):
        spec = scenegen.SceneSpec(p=5, q=24, H=42, W=40, r_a=1, r_b=4, n_targets=4, snr_db=(0.0, 15.0), block=20)
        base = dict(p=5, q=24, n=256, r_a=1, r_b=4)
    else:
        spec = scenegen.SceneSpec(p=6, q=16, H=36, W=40, r_a=2, r_b=3, n_targets=4)
        base = dict(p=6, q=16, n=200, r_a=2, r_b=3)
    return spec, scenegen.BASE_SEED + 70 + len(case), base, prec


# ------------------------------------------- one case per remaining kernel class
# Kernel classes are (p, q, r_b bound, precision) with r_b bound 4 (r_b <= 4)
# or 8 (5 <= r_b <= 8).  These frames reach the classes that no other parity
# case reaches, among them every class the uneven-tile batches can draw
# (p = 3, q in {8, 12, 16}, r_a in {1, 2}, r_b in {2..6}, both precisions).
CLASSES = {
    # name: (p, q, n, r_a, r_b, precision, side)
    "fp32_p2q8": (2, 8, 64, 1, 3, "fp32", 64),
    "fp32_p2q16": (2, 16, 128, 1, 4, "fp32", 64),
    "fp32_p3q8_rb6_ra2": (3, 8, 64, 2, 6, "fp32", 72),
    "fp32_p3q12_rb4_ra2": (3, 12, 128, 2, 4, "fp32", 72),
    "fp32_p3q16_rb5_ra2": (3, 16, 200, 2, 5, "fp32", 80),
    "fp32_p4q16_ra2": (4, 16, 256, 2, 4, "fp32", 64),
    "fp32_p6q8_ra2": (6, 8, 128, 2, 3, "fp32", 64),
    "bf16x3_p3q12_rb3": (3, 12, 128, 1, 3, "bf16x3", 72),
    "bf16x3_p3q16_rb6_ra2": (3, 16, 256, 2, 6, "bf16x3", 80),
    "fp32_f64_p3q8": (3, 8, 64, 1, 3, "fp32_f64", 64),
    "fp32_f64_p3q16_ra2": (3, 16, 200, 2, 4, "fp32_f64", 72),
}


def class_case(name):
    p, q, n, ra, rb, prec, side = CLASSES[name]
    spec = scenegen.SceneSpec(p=p, q=q, H=side, W=side + 5, r_a=ra, r_b=rb, n_targets=5, snr_db=(0.0, 15.0),
                              block=24)
    return spec, scenegen.BASE_SEED + 300 + sum(map(ord, name)), dict(p=p, q=q, n=n, r_a=ra, r_b=rb), prec


# --------------------------------------------- strong scatterers (sliding window)
# Point scatterers placed so that they enter and leave the training windows of
# pixels in the middle of sliding-window chains; the strongest is 40-60 dB
# above the noise floor (10-30 dB above the 30 dB clutter), the other two 10
# and 20 dB below it.
HDR = {
    # name: (p, q, n, r_b, precision, side, strongest scatterer in dB over the noise)
    "fp32_p3q16_40db": (3, 16, 200, 4, "fp32", 72, 40.0),
    "fp32_p3q8_40db": (3, 8, 64, 3, "fp32", 56, 40.0),
    "fp32_p5q24_40db": (5, 24, 256, 4, "fp32", 44, 40.0),
    "bf16x3_p3q16_40db": (3, 16, 200, 4, "bf16x3", 72, 40.0),
    "bf16x3_p3q16_50db": (3, 16, 200, 4, "bf16x3", 72, 50.0),
    "fp32_p3q16_60db": (3, 16, 200, 4, "fp32", 72, 60.0),
    "fp32_p3q8_60db": (3, 8, 64, 3, "fp32", 56, 60.0),
    "fp32_p5q24_60db": (5, 24, 256, 4, "fp32", 44, 60.0),
    "bf16x3_p3q16_60db": (3, 16, 200, 4, "bf16x3", 72, 60.0),
    # FP32 covariance (full sums) with FP64 solves, on the FP32 cases' scenes
    "fp32_f64_p3q16_50db": (3, 16, 200, 4, "fp32_f64", 72, 50.0),
    "fp32_f64_p3q16_60db": (3, 16, 200, 4, "fp32_f64", 72, 60.0),
    "fp32_f64_p3q8_60db": (3, 8, 64, 3, "fp32_f64", 56, 60.0),
}
# cases that reuse another precision's scene (same seed and scatterers)
HDR_SAME_SCENE = {
    "fp32_f64_p3q16_50db": "fp32_p3q16_60db",
    "fp32_f64_p3q16_60db": "fp32_p3q16_60db",
    "fp32_f64_p3q8_60db": "fp32_p3q8_60db",
}
# (row, col) as fractions of the frame, dB below the case's strongest scatterer
HDR_SCATTERERS = ((0.55, 0.45, 0.0), (0.3, 0.7, 10.0), (0.75, 0.25, 20.0))
# Accuracy envelope, measured on the GPU against the oracle on scenes like
# these (frame pass with the sliding window, and the probe's full sums, which
# err alike, so the sliding window is not what limits them):
#   plain FP32 path (FP32 covariance and solves): max error 1.4e-5 at 40 dB,
#     1.5e-4 - 3.2e-4 at 50 dB, 1.5e-3 - 6.2e-1 at 60 dB;
#   mixed path (split-BF16 covariance, FP64 solves): 2.7e-6 at 40 dB,
#     3.7e-5 - 5.9e-3 at 50 dB (scene-dependent, and on one scene moved
#     from 5.9e-3 to 7.9e-5 by last-place changes in the FP32 sweep scale
#     factors), 1.9e-3 at 60 dB (3.8e-3 - 1.9e-2 with the earlier
#     200-step cap on the time-subspace iteration).  Its products resolve about 2^-17 of each
#     product; an FP64 emulation of exactly that split puts the 60 dB error
#     at 1.8e-3 from the covariance alone.
#   FP32 covariance (full sums) with FP64 solves: within 1e-4 at 50 dB and on
#     the q = 8 scene at 60 dB; on the q = 16 scene at 60 dB the 99th
#     percentile is 1.6e-5 and the worst pixel 7.8e-3.
# Near a 60 dB scatterer the r_b-th and next eigenvalues of B-hat come within
# a few per cent of each other (ratio 0.95 - 0.99), where subspace iteration
# needs hundreds to ~1 500 steps; the FP64 solves now allow 4 000 (they
# stopped at 200 and left those pixels at up to 7.2e-2, mixed path 1.9e-2).
# Both paths hold the 1e-4 bar up to 40 dB over the noise (10 dB over the
# clutter), the FP32 / FP64 form up to 50 dB.  The mixed 50 dB case straddles it and is graded against its
# envelope's bound; the 60 dB cases are expected to fail the bar.
HDR_ENVELOPE_TOL = {
    "bf16x3_p3q16_50db": 1e-2,
}
HDR_OUTSIDE_ENVELOPE = {
    "fp32_p3q16_60db": "FP32 covariance and eigensolves resolve 60 dB scatterers to about 1e-1 - 6e-1 (FP32 envelope: 40 dB)",
    "fp32_p3q8_60db": "FP32 covariance and eigensolves resolve 60 dB scatterers to about 2e-3 (FP32 envelope: 40 dB)",
    "fp32_p5q24_60db": "FP32 covariance and eigensolves resolve 60 dB scatterers to about 1e-1 (FP32 envelope: 40 dB)",
    "bf16x3_p3q16_60db": "split-BF16 products resolve ~2^-17 of a product: a 60 dB scatterer gives 1.9e-3, the "
                         "level an FP64 emulation of the split covariance alone reaches (mixed envelope: 40 dB)",
    "fp32_f64_p3q16_60db": "with a 60 dB scatterer the worst pixel misses the bar at 1.34e-4 (p99 1.6e-5), once "
                           "the stop-rule tie at (22, 44) is graded against the oracle at the GPU's iteration "
                           "count (FP32-covariance / FP64-solve envelope: 50 dB)",
}


def hdr_case(name):
    p, q, n, rb, prec, side, top = HDR[name]
    spec = scenegen.SceneSpec(p=p, q=q, H=side, W=side, r_a=1, r_b=rb, n_targets=3, snr_db=(5.0, 15.0))
    stem = HDR_SAME_SCENE.get(name, name).rsplit("_", 1)[0]   # the same scene at every scatterer strength
    return spec, scenegen.BASE_SEED + 400 + len(stem), dict(p=p, q=q, n=n, r_a=1, r_b=rb), prec


def hdr_scene(name):
    """The case's scene with its strong scatterers added (Eq. (8) returns with
    |alpha|^2 = 10^(dB/10) per element, random spatial phase)."""
    spec, seed, base, prec = hdr_case(name)
    sc = scenegen.make_scene(spec, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    pos = []
    top = HDR[name][6]
    for fr, fc, below in HDR_SCATTERERS:
        db = top - below
        r, c = int(fr * spec.H), int(fc * spec.W)
        theta = rng.uniform(0.0, 2.0 * np.pi)
        amp = np.sqrt(10.0 ** (db / 10.0)) * np.exp(1j * rng.uniform(0.0, 2.0 * np.pi))
        sc.x[:, r, c, :] += (amp * np.outer(np.exp(1j * theta * np.arange(spec.p)), np.ones(spec.q))).astype(
            np.complex64)
        pos.append((r, c))
    return sc, np.array(pos), base, prec


def all_frame_cases():
    """Every whole-frame parity case: name -> (spec, seed, base, precision)."""
    out = {}
    out["tiny"] = (scenegen.TINY, scenegen.BASE_SEED, dict(p=3, q=8, n=64, r_a=1, r_b=3), "fp32")
    for H, W in ((80, 80), (37, 53)):
        out[f"frame_{H}x{W}"] = (
            scenegen.SceneSpec(p=3, q=16, H=H, W=W, r_a=1, r_b=4, n_targets=8, snr_db=(0.0, 15.0), block=32),
            scenegen.BASE_SEED + 11, dict(p=3, q=16, n=200, r_a=1, r_b=4), "fp32")
    for c in VARIANTS:
        out["variant_" + c] = variant_case(c)
    for c in MIXED:
        out["mixed_" + c] = mixed_case(c)
    for c in WIDE:
        out["wide_" + c] = wide_case(c)
    for c in CLASSES:
        out["class_" + c] = class_case(c)
    return out
