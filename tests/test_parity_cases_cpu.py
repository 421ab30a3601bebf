"""CPU checks of the GPU parity cases (oracle only, no GPU).

  * Every whole-frame case grades at least 80 % of its valid pixels (the
    truncation-gap rule: pixels where several subspaces are correct are not
    graded), so no GPU parity test can pass on an empty or tiny graded set.
    Checked on a seeded sample of 300 valid pixels per case (plus the
    targets), which keeps the CPU suite short.
  * The cases reach every kernel class that the library's instantiation
    tables build, and every class that the uneven-tile batches can draw.
"""
import os
import re

import numpy as np
import pytest

import oracle
import scenegen
from tests import parity_cases as pc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_03622_amd", "csrc")
MIN_GRADED = 0.8


def graded_fraction(x, base, extra=None, count=300):
    cfg = oracle.OracleConfig(**{k: v for k, v in base.items() if k != "stat_mode"},
                              stat_mode=base.get("stat_mode", "glrt"))
    H, W = x.shape[1], x.shape[2]
    region = oracle.valid_region(H, W, cfg.training_stencil())
    if region[0] == region[1] or region[2] == region[3]:
        return 0, 0
    pix = scenegen.random_pixels(H, W, count, 5, region=region)
    if extra is not None:
        pix = np.concatenate([pix, np.asarray(extra, np.int32).reshape(-1, 2)])
    out = oracle.kron_stap_pixels(x, pix, cfg)
    out["T"] = np.where(out["valid"], out["T"], np.nan)
    ga = oracle.relative_gaps(out["lam_A"], cfg.r_a)
    gb = oracle.relative_gaps(out["lam_B"], cfg.r_b)
    finite = np.isfinite(out["T"])
    g = finite & (ga >= 1e-3) & (gb >= 1e-3)
    return int(g.sum()), int(finite.sum())


CASES = pc.all_frame_cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_case_grades_most_valid_pixels(name):
    spec, seed, base, _ = CASES[name]
    sc = scenegen.make_scene(spec, seed=seed)
    graded, valid = graded_fraction(sc.x, base, sc.targets)
    assert valid > 0, f"{name}: no valid pixel"
    assert graded >= MIN_GRADED * valid, f"{name}: graded {graded}/{valid}"


@pytest.mark.parametrize("name", sorted(pc.HDR))
def test_strong_scatterer_case_grades_most_valid_pixels(name):
    sc, pos, base, _ = pc.hdr_scene(name)
    graded, valid = graded_fraction(sc.x, base, pos)
    assert valid > 0 and graded >= MIN_GRADED * valid, f"{name}: graded {graded}/{valid}"


def built_classes():
    """(p, q, r_b bound, precision) of every kernel in the instantiation tables."""
    out = set()
    for f in ("kstap_kern_fp32.hip", "kstap_kern_bf16.hip", "kstap_kern_wide.hip", "kstap_kern_f32f64.hip"):
        txt = open(os.path.join(CSRC, f)).read()
        for m in re.finditer(r"KSTAP_ENTRY\((\d+),\s*(\d+),\s*(\d+),\s*(\d+)\)", txt):
            if "#define" in txt[max(0, m.start() - 8):m.start()]:
                continue
            out.add(tuple(int(v) for v in m.groups()))
        for m in re.finditer(r"\{(\d+),\s*(\d+),\s*(\d+),\s*(\d+),\s*(?:true|false)", txt):
            out.add(tuple(int(v) for v in m.groups()))
    return out


def reached_classes():
    prec = {"fp32": 0, "bf16x3": 1, "fp32_f64": 2}
    out = set()
    for spec, seed, base, pr in CASES.values():
        out.add((base["p"], base["q"], 4 if base["r_b"] <= 4 else 8, prec[pr]))
    for name in pc.HDR:
        _, _, base, pr = pc.hdr_case(name)
        out.add((base["p"], base["q"], 4 if base["r_b"] <= 4 else 8, prec[pr]))
    return out


def test_cases_reach_every_built_kernel_class():
    built = built_classes()
    assert len(built) >= 20
    missing = sorted(built - reached_classes())
    assert not missing, f"kernel classes without a parity case: {missing}"


def test_cases_reach_every_batch_class():
    """Tiles of the uneven batches: p = 3, q in {8, 12, 16}, r_b in {2..6},
    both precisions (the batch tile generator's ranges)."""
    specs = scenegen.batch_tile_specs()
    drawn = {(3, sp.q, 4 if sp.r_b <= 4 else 8, pr) for sp, _ in specs for pr in (0, 1)}
    assert drawn <= reached_classes()
    assert drawn <= built_classes()
