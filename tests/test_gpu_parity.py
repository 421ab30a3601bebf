"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (per pixel, on graded pixels):
  err = |T_gpu - T_ref| / max(T_ref, 1) <= 1e-4, where graded pixels are the
  valid pixels whose truncation gaps (lambda_r - lambda_{r+1}) / lambda_1 are
  >= 1e-3 for both factors (elsewhere several subspaces are correct);
  detection maps identical outside the margin band |T_ref - tau| <= 1e-3 tau.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle
import scenegen
from tests import parity_cases as pc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4

_gspec = importlib.util.spec_from_file_location(
    "make_golden", os.path.join(os.path.dirname(__file__), "golden", "make_golden.py"))
golden = importlib.util.module_from_spec(_gspec)
_gspec.loader.exec_module(golden)


def _kstap():
    import paper_1604_03622_amd as kstap
    return kstap


def dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch.device("cuda:0")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev())


def graded_mask(ref, r_a, r_b):
    ga = oracle.relative_gaps(ref["lam_A"], r_a)
    gb = oracle.relative_gaps(ref["lam_B"], r_b)
    return ref["valid"] & np.isfinite(ref["T"]) & (ga >= 1e-3) & (gb >= 1e-3)


def rel_err(tg, tr):
    return np.abs(tg - tr) / np.maximum(np.abs(tr), 1.0)


def check_parity(Tg, Dg, ref, tau, r_a, r_b, label, min_graded=0.8, tol=None):
    """Grades T and D against the oracle; fails if no pixel, or fewer than
    `min_graded` of the valid pixels with a finite T, are graded.  `tol`
    (default: the 1e-4 bar) bounds the relative error of T; detections must
    agree outside a margin band of 10 tol around the threshold."""
    tol = TOL if tol is None else tol
    Tg = np.asarray(Tg, dtype=np.float64)
    g = graded_mask(ref, r_a, r_b)
    base = ref["valid"] & np.isfinite(ref["T"])
    assert g.any(), f"{label}: no pixel graded"
    assert g.sum() >= min_graded * base.sum(), f"{label}: only {int(g.sum())}/{int(base.sum())} valid pixels graded"
    e = rel_err(Tg, ref["T"])
    worst = float(e[g].max())
    note(f"[{label}] graded {int(g.sum())}/{int(base.sum())} max err {worst:.3e} p99 "
         f"{float(np.quantile(e[g], 0.99)):.3e}")
    assert worst <= tol, f"{label}: max relative error {worst:.3e} > {tol}"
    band = np.abs(ref["T"] - tau) <= 10 * tol * tau
    outside = g & ~band
    mism = np.nonzero(Dg[outside] != ref["D"][outside])[0]
    assert mism.size == 0, f"{label}: {mism.size} detection mismatches outside the margin band"
    # outside the valid region everything is zero
    assert np.all(Tg[~ref["valid"]] == 0.0)
    assert np.all(Dg[~ref["valid"]] == 0)


def run_frame(plan, x):
    kstap = _kstap()
    xd = to_dev(x)
    T, D = kstap.run(plan, xd)
    torch.cuda.synchronize()
    return T.cpu().numpy(), D.cpu().numpy(), xd


def frame_oracle(x, cfg):
    out = oracle.kron_stap_frame(x, cfg)
    H, W = x.shape[1], x.shape[2]
    ref = dict(T=out["T_img"].ravel(), D=out["D_img"].ravel())
    valid = np.zeros((H, W), bool)
    lam_A = np.zeros((H * W, cfg.p))
    lam_B = np.zeros((H * W, cfg.q))
    idx = out["pixels"][:, 0] * W + out["pixels"][:, 1]
    valid.ravel()[idx] = True
    lam_A[idx] = out["lam_A"]
    lam_B[idx] = out["lam_B"]
    ref.update(valid=valid.ravel(), lam_A=lam_A, lam_B=lam_B)
    return ref, out


# ------------------------------------------------------------------ frames
@pytest.mark.parametrize("name", sorted(golden.FIXTURES))
def test_golden_fixture_parity(name):
    """The HIP path against the oracle outputs stored under tests/golden/:
    T from a whole-frame run and eta / iterations from the probe, at the
    stored pixels (targets, valid-region corners, a seeded sample)."""
    kstap = _kstap()
    spec, seed, base, _, _ = golden.FIXTURES[name]
    head, t = golden.read(name)
    sc = scenegen.make_scene(spec, seed=seed)
    assert head["x_sha256"] == golden.scene_sha256(sc.x), "scene generator changed"
    plan = kstap.Plan(**base)
    assert plan.tau == pytest.approx(float(head["tau"]), rel=1e-9)
    pix = np.stack([t["r"], t["c"]], 1).astype(np.int32)
    note(f"golden {name}: frame {spec.H}x{spec.W} and probe of {pix.shape[0]} px")
    Tg, Dg, xd = run_frame(plan, sc.x)
    pr = kstap.probe(plan, xd, pix)
    torch.cuda.synchronize()
    T_at = Tg[pix[:, 0], pix[:, 1]].astype(np.float64)
    D_at = Dg[pix[:, 0], pix[:, 1]]
    valid = t["iters"] > 0
    g = valid & (t["gap_A"] >= 1e-3) & (t["gap_B"] >= 1e-3)
    assert g.sum() >= 0.8 * g.size - 6
    e = rel_err(T_at, t["T"])
    note(f"[golden {name}] graded {int(g.sum())}/{g.size} max err {e[g].max():.3e}")
    assert e[g].max() <= TOL
    band = np.abs(t["T"] - plan.tau) <= 1e-3 * plan.tau
    assert np.array_equal(D_at[g & ~band], t["D"][g & ~band])
    assert np.all(T_at[~valid] == 0) and np.all(D_at[~valid] == 0)
    it = pr["iters"].cpu().numpy()
    eta = pr["eta"].cpu().numpy()
    assert np.all(np.abs(it[g] - t["iters"][g]) <= 1)
    assert np.allclose(eta[g], t["eta"][g], rtol=1e-3, atol=1e-6)
    assert np.all(it[~valid] == 0)


def test_tiny_frame_full_parity():
    """64 x 64, p=3, q=8, n=64 (10 x 10 window minus 3 x 3 guard), r_a=1, r_b=3."""
    kstap = _kstap()
    sc = scenegen.make_scene(scenegen.TINY)
    cfg = oracle.OracleConfig(p=3, q=8, n=64, r_a=1, r_b=3)
    plan = kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3)
    note("tiny frame 64x64 p3 q8 n64")
    Tg, Dg, _ = run_frame(plan, sc.x)
    ref, _ = frame_oracle(sc.x, cfg)
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, 1, 3, "tiny")


@pytest.mark.parametrize("H,W", [(80, 80), (37, 53)])
def test_full_frame_shape_parity(H, W):
    """p=3, q=16, n=200 (16 x 16 window), rotating factors, ragged sizes."""
    kstap = _kstap()
    spec = scenegen.SceneSpec(p=3, q=16, H=H, W=W, r_a=1, r_b=4, n_targets=8, snr_db=(0.0, 15.0), block=32)
    sc = scenegen.make_scene(spec, seed=scenegen.BASE_SEED + 11)
    cfg = oracle.OracleConfig(p=3, q=16, n=200, r_a=1, r_b=4)
    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4)
    note(f"frame {H}x{W} p3 q16 n200")
    Tg, Dg, _ = run_frame(plan, sc.x)
    ref, _ = frame_oracle(sc.x, cfg)
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, 1, 4, f"{H}x{W}")


_FULL_SIZE = {
    # name: (scene, plan / oracle configuration, precision, random pixels)
    "full_frame_fp32": (scenegen.FULL_FRAME, dict(p=3, q=16, n=200, r_a=1, r_b=4), "fp32", 1500),
    "full_frame_bf16x3": (scenegen.FULL_FRAME, dict(p=3, q=16, n=200, r_a=1, r_b=4), "bf16x3", 1500),
    "mixed_fp32": (scenegen.MIXED, dict(p=5, q=24, n=256, r_a=1, r_b=4), "fp32", 600),
    "mixed_bf16x3": (scenegen.MIXED, dict(p=5, q=24, n=256, r_a=1, r_b=4), "bf16x3", 600),
}
_scene_cache = {}


def _full_size_scene(spec):
    # the two precisions of a workload share its scene (generating the
    # 2048 x 2048 frame takes a while); only the latest scene is kept
    if spec not in _scene_cache:
        _scene_cache.clear()
        _scene_cache[spec] = scenegen.make_scene(spec)
    return _scene_cache[spec]


@pytest.mark.parametrize("case", list(_FULL_SIZE))
def test_full_size_frame_sampled_parity(case):
    """The benchmarked workloads at full size, the whole frame in one launch as
    the benchmark runs it: 2048 x 2048, p=3, q=16, n=200 and 1024 x 1024,
    p=5, q=24, n=256, in both precisions, checked on seeded pixels plus every
    target and the corners of the frame and of its valid region."""
    kstap = _kstap()
    spec, base, prec, count = _FULL_SIZE[case]
    sc = _full_size_scene(spec)
    cfg = oracle.OracleConfig(**base)
    plan = kstap.Plan(**base, precision=prec)
    H, W = spec.H, spec.W
    note(f"full size {case}: {H}x{W} p{base['p']} q{base['q']} n{base['n']} {prec}")
    Tg, Dg, _ = run_frame(plan, sc.x)
    region = oracle.valid_region(H, W, cfg.training_stencil())
    pix = np.concatenate([scenegen.random_pixels(H, W, count, 7, region=region), sc.targets,
                          np.array([[0, 0], [H - 1, W - 1], [region[0], region[2]], [region[1] - 1, region[3] - 1]])])
    ref = oracle.kron_stap_pixels(sc.x, pix, cfg)
    check_parity(Tg[pix[:, 0], pix[:, 1]], Dg[pix[:, 0], pix[:, 1]], ref, plan.tau, base["r_a"], base["r_b"],
                 f"{case} sampled")
    assert np.isfinite(Tg).all()
    r0, r1, c0, c1 = region
    inner = np.zeros_like(Tg, bool)
    inner[r0:r1, c0:c1] = True
    assert np.all(Tg[~inner] == 0) and np.all(Dg[~inner] == 0)


# ------------------------------------------------------------------- probe
def test_probe_subspaces_and_iterations():
    kstap = _kstap()
    sc = scenegen.make_scene(scenegen.TINY)
    cfg = oracle.OracleConfig(p=3, q=8, n=64, r_a=1, r_b=3)
    plan = kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3)
    pix = np.concatenate([scenegen.random_pixels(64, 64, 200, 3), sc.targets])
    xd = to_dev(sc.x)
    note("probe tiny 205 px")
    pr = kstap.probe(plan, xd, pix)
    T_run, _ = kstap.run(plan, xd)
    torch.cuda.synchronize()
    ref = oracle.kron_stap_pixels(sc.x, pix, cfg)
    g = ref["valid"] & (oracle.relative_gaps(ref["lam_B"], 3) >= 1e-3)
    T_probe = pr["T"].cpu().numpy()
    assert rel_err(T_probe[g], ref["T"][g]).max() <= TOL
    # the probe runs the frame pass's body on single pixels; the frame pass
    # may update the previous pixel's covariance instead of summing all n
    # vectors, which changes only the FP32 summation order
    assert rel_err(T_probe, T_run.cpu().numpy()[pix[:, 0], pix[:, 1]]).max() <= 2e-5
    UA = pr["U_A"].cpu().numpy().astype(np.complex128)
    UB = pr["U_B"].cpu().numpy().astype(np.complex128)
    PA = UA @ np.conj(np.swapaxes(UA, 1, 2))
    PB = UB @ np.conj(np.swapaxes(UB, 1, 2))
    PA_ref = ref["U_A"] @ np.conj(np.swapaxes(ref["U_A"], 1, 2))
    PB_ref = ref["U_B"] @ np.conj(np.swapaxes(ref["U_B"], 1, 2))
    da = np.abs(PA - PA_ref).max(axis=(1, 2))[g]
    db = np.abs(PB - PB_ref).max(axis=(1, 2))[g]
    note(f"probe projector distance max A {da.max():.2e} B {db.max():.2e}")
    assert da.max() <= 1e-4 and db.max() <= 1e-4
    # orthonormal bases
    eye = np.abs(np.conj(np.swapaxes(UB, 1, 2)) @ UB - np.eye(3)).max(axis=(1, 2))[g]
    assert eye.max() <= 1e-5
    it_g = pr["iters"].cpu().numpy()[g]
    assert np.all(np.abs(it_g - ref["iters"][g]) <= 1)
    eta_g = pr["eta"].cpu().numpy()[g]
    assert np.allclose(eta_g, ref["eta"][g], rtol=1e-3, atol=1e-6)
    # pixels outside the valid region
    outside = ~ref["valid"]
    assert np.all(T_probe[outside] == 0) and np.all(pr["iters"].cpu().numpy()[outside] == 0)


# -------------------------------------------------------------- edge cases
def test_edge_zero_nan_and_too_small_frames():
    kstap = _kstap()
    plan = kstap.Plan(p=3, q=8, n=64, r_a=1, r_b=3)
    note("edge: zero frame")
    Tg, Dg, _ = run_frame(plan, np.zeros((3, 30, 30, 8), np.complex64))
    assert np.all(Tg == 0) and np.all(Dg == 0)
    note("edge: frame smaller than the stencil")
    Tg, Dg, _ = run_frame(plan, scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=9, W=12, n_targets=0), 5).x)
    assert np.all(Tg == 0) and np.all(Dg == 0)
    note("edge: 1 x 1 frame")
    Tg, Dg, _ = run_frame(plan, np.ones((3, 1, 1, 8), np.complex64))
    assert Tg.shape == (1, 1) and Tg[0, 0] == 0
    note("edge: NaN sample")
    x = scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=30, W=30, n_targets=0), 6).x
    x[1, 15, 15, 2] = np.nan
    Tg, Dg, _ = run_frame(plan, x)
    cfg = oracle.OracleConfig(p=3, q=8, n=64, r_a=1, r_b=3)
    ref, _ = frame_oracle(x, cfg)
    nan_ref = np.isnan(ref["T"])
    assert np.array_equal(np.isnan(Tg.ravel()), nan_ref)
    assert np.all(Dg.ravel()[nan_ref] == 0)
    check_parity(np.where(nan_ref, 0, Tg.ravel()), Dg.ravel(), dict(ref, T=np.where(nan_ref, 0, ref["T"])),
                 plan.tau, 1, 3, "nan-frame", min_graded=0.6)


def oracle_cfg(base):
    return oracle.OracleConfig(**{k: v for k, v in base.items() if k != "stat_mode"},
                               stat_mode=base.get("stat_mode", "glrt"))


@pytest.mark.parametrize("case", pc.VARIANTS)
def test_configuration_variants(case):
    kstap = _kstap()
    spec, seed, base, prec = pc.variant_case(case)
    sc = scenegen.make_scene(spec, seed=seed)
    plan = kstap.Plan(**base, precision=prec)
    note(f"variant {case}")
    Tg, Dg, _ = run_frame(plan, sc.x)
    ref, _ = frame_oracle(sc.x, oracle_cfg(base))
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, base["r_a"], base["r_b"], case)


@pytest.mark.parametrize("name", sorted(pc.CLASSES))
def test_kernel_class_parity(name):
    """One whole frame per kernel class that no other case reaches (among
    them every class of the uneven-tile batches: q in {8, 12, 16} with
    r_b <= 4 or 5..8, FP32 and split BF16), against the oracle element by
    element, plus probe subspaces on a sample of its pixels."""
    kstap = _kstap()
    spec, seed, base, prec = pc.class_case(name)
    sc = scenegen.make_scene(spec, seed=seed)
    plan = kstap.Plan(**base, precision=prec)
    note(f"class {name}: {spec.H}x{spec.W} {base} {prec}")
    Tg, Dg, xd = run_frame(plan, sc.x)
    ref, out = frame_oracle(sc.x, oracle_cfg(base))
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, base["r_a"], base["r_b"], "class " + name)
    sel = np.arange(0, len(out["pixels"]), 11)
    pr = kstap.probe(plan, xd, out["pixels"][sel])
    torch.cuda.synchronize()
    g = graded_mask(dict(T=out["T"][sel], lam_A=out["lam_A"][sel], lam_B=out["lam_B"][sel],
                         valid=np.ones(sel.size, bool)), base["r_a"], base["r_b"])
    UA = pr["U_A"].cpu().numpy().astype(np.complex128)
    UB = pr["U_B"].cpu().numpy().astype(np.complex128)
    dA = np.abs(UA @ np.conj(np.swapaxes(UA, 1, 2)) - out["U_A"][sel] @ np.conj(np.swapaxes(out["U_A"][sel], 1, 2)))
    dB = np.abs(UB @ np.conj(np.swapaxes(UB, 1, 2)) - out["U_B"][sel] @ np.conj(np.swapaxes(out["U_B"][sel], 1, 2)))
    dA, dB = dA.max(axis=(1, 2))[g], dB.max(axis=(1, 2))[g]
    note(f"[class {name}] probe projector distance A {dA.max():.2e} B {dB.max():.2e} over {int(g.sum())} px")
    assert dA.max() <= 1e-4 and dB.max() <= 1e-4


def regrade_stop_ties(kstap, plan, xd, Tg, ref, out, cfg, tol):
    """Where several results are correct: LR-Kron stops at the first k with
    |eta_k - eta_{k-1}| <= eps (Sec. 4, Algorithm 2), and where that test
    lands within 0.1 % of eps the GPU (eta from its own covariance) may stop
    one iteration earlier or later.  For such a graded pixel whose T misses
    the bar and whose GPU iteration count (from the probe) differs from the
    oracle's by one, the reference becomes the oracle run to the GPU's count.
    Returns the reference T and the number of pixels re-graded."""
    H, W = Tg.shape
    T = ref["T"].copy()
    g = graded_mask(ref, cfg.r_a, cfg.r_b)
    bad = np.nonzero(g & (rel_err(Tg.ravel(), ref["T"]) > tol))[0]
    if bad.size == 0 or bad.size > 64:
        return T, 0
    pix = np.stack([bad // W, bad % W], 1).astype(np.int32)
    pr = kstap.probe(plan, xd, pix)
    torch.cuda.synchronize()
    kg = pr["iters"].cpu().numpy()
    where = {(int(r), int(c)): i for i, (r, c) in enumerate(out["pixels"])}
    st = cfg.training_stencil()
    b_s = cfg.temporal_steering()
    n = 0
    for j, f in enumerate(bad):
        r, c = int(pix[j, 0]), int(pix[j, 1])
        ko = int(out["iters"][where[(r, c)]])
        if abs(int(kg[j]) - ko) != 1:
            continue
        k = min(ko, int(kg[j]))
        S = oracle.sample_covariance(xd.cpu().numpy(), np.array([r]), np.array([c]), st)
        R = oracle.rearrange(S, cfg.p, cfg.q)
        e1 = oracle.lr_kron(R, cfg.p, cfg.q, cfg.r_a, cfg.r_b, 0.0, k - 1, k - 1)["eta"][0]
        e2 = oracle.lr_kron(R, cfg.p, cfg.q, cfg.r_a, cfg.r_b, 0.0, k, k)["eta"][0]
        if abs(abs(e2 - e1) - cfg.eps) > 1e-3 * cfg.eps:
            continue
        est = oracle.lr_kron(R, cfg.p, cfg.q, cfg.r_a, cfg.r_b, 0.0, int(kg[j]), int(kg[j]))
        Xt = oracle.snapshots(xd.cpu().numpy(), np.array([r]), np.array([c]))
        T[f] = oracle.kron_stap_statistic(Xt, est["U_A"], est["U_B"], b_s)[0]
        note(f"  stop-rule tie at ({r}, {c}): |d eta| {abs(e2 - e1):.4e} at k = {k}, oracle {ko} vs GPU "
             f"{int(kg[j])} iterations; T {Tg[r, c]:.6g} against the oracle at {int(kg[j])}: {T[f]:.6g}")
        n += 1
    return T, n


@pytest.mark.parametrize("name", [
    pytest.param(n, marks=pytest.mark.xfail(strict=True, reason=pc.HDR_OUTSIDE_ENVELOPE[n]))
    if n in pc.HDR_OUTSIDE_ENVELOPE else n for n in sorted(pc.HDR)])
def test_strong_scatterers_sliding_window(name):
    """Point scatterers 40-60 dB above the noise enter and leave the training
    windows of pixels in the middle of sliding-window chains: inside each
    path's accuracy envelope the frame pass (covariances updated from the
    previous pixel's) matches the oracle at the 1e-4 bar on every graded
    pixel, and the probe (every covariance summed from scratch) within the
    same bar at the pixels whose windows hold a scatterer.  A case at the
    edge of its path's envelope is graded against the envelope's bound."""
    kstap = _kstap()
    tol = pc.HDR_ENVELOPE_TOL.get(name, TOL)
    sc, pos, base, prec = pc.hdr_scene(name)
    plan = kstap.Plan(**base, precision=prec)
    H, W = sc.x.shape[1], sc.x.shape[2]
    note(f"strong scatterers {name}: {H}x{W} {base} {prec}")
    Tg, Dg, xd = run_frame(plan, sc.x)
    ref, out = frame_oracle(sc.x, oracle_cfg(base))
    T_tie, nties = regrade_stop_ties(kstap, plan, xd, Tg, ref, out, oracle_cfg(base), tol)
    moved = T_tie != ref["T"]
    ref["D"] = np.where(moved, (T_tie > plan.tau).astype(ref["D"].dtype), ref["D"])
    ref["T"] = T_tie
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, base["r_a"], base["r_b"], "hdr " + name, tol=tol)
    # pixels whose windows held a scatterer, and their neighbours in the chain
    st = plan.stencil
    near = set()
    for r, c in pos:
        for dr, dc in st:
            near.add((int(r - dr), int(c - dc)))
    r0, r1, c0, c1 = plan.valid_region(H, W)
    sel = np.array(sorted(p for p in near if r0 <= p[0] < r1 and c0 <= p[1] < c1), np.int32)
    pr = kstap.probe(plan, xd, sel)
    torch.cuda.synchronize()
    eP = rel_err(pr["T"].cpu().numpy(), Tg[sel[:, 0], sel[:, 1]]).max()
    note(f"[hdr {name}] probe vs frame over {len(sel)} px whose windows hold a scatterer: {eP:.2e}")
    assert eP <= tol


def test_repeatable_bitwise():
    kstap = _kstap()
    sc = scenegen.make_scene(scenegen.SceneSpec(p=3, q=16, H=48, W=48, r_b=4, n_targets=3), 9)
    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4)
    xd = to_dev(sc.x)
    note("repeatability")
    T1, _ = kstap.run(plan, xd)
    T2, _ = kstap.run(plan, xd)
    torch.cuda.synchronize()
    assert torch.equal(T1, T2)


# -------------------------------------------------------- mixed precision
@pytest.mark.parametrize("case", pc.MIXED)
def test_mixed_precision_parity(case):
    """Split-BF16 covariance (three products, FP32 accumulation) with FP64
    eigensolves and statistic, against the FP64 oracle at the same 1e-4 bar;
    per-output errors (T, U_A and U_B projectors, eta, iterations) reported."""
    kstap = _kstap()
    spec, seed, base, _ = pc.mixed_case(case)
    sc = scenegen.make_scene(spec, seed=seed)
    plan = kstap.Plan(**base, precision="bf16x3")
    ocfg = oracle_cfg(base)
    note(f"mixed {case}")
    Tg, Dg, xd = run_frame(plan, sc.x)
    ref, out = frame_oracle(sc.x, ocfg)
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, base["r_a"], base["r_b"], "bf16x3 " + case)
    # per-output report on the valid pixels through the probe
    pix = out["pixels"]
    pr = kstap.probe(plan, xd, pix)
    torch.cuda.synchronize()
    g = graded_mask(dict(T=out["T"], lam_A=out["lam_A"], lam_B=out["lam_B"], valid=np.ones(len(pix), bool)),
                    base["r_a"], base["r_b"])
    UA = pr["U_A"].cpu().numpy().astype(np.complex128)
    UB = pr["U_B"].cpu().numpy().astype(np.complex128)
    dA = np.abs(UA @ np.conj(np.swapaxes(UA, 1, 2)) - out["U_A"] @ np.conj(np.swapaxes(out["U_A"], 1, 2))).max(axis=(1, 2))
    dB = np.abs(UB @ np.conj(np.swapaxes(UB, 1, 2)) - out["U_B"] @ np.conj(np.swapaxes(out["U_B"], 1, 2))).max(axis=(1, 2))
    eT = rel_err(pr["T"].cpu().numpy().astype(np.float64), out["T"])
    eeta = np.abs(pr["eta"].cpu().numpy() - out["eta"]) / np.maximum(out["eta"], 1e-12)
    it = np.abs(pr["iters"].cpu().numpy() - out["iters"])
    note(f"[bf16x3 {case}] per-output max error over {int(g.sum())} graded px: T {eT[g].max():.2e}, "
         f"P_A {dA[g].max():.2e}, P_B {dB[g].max():.2e}, eta(rel) {eeta[g].max():.2e}, iters diff {it[g].max()}")
    assert eT[g].max() <= TOL and dA[g].max() <= 1e-4 and dB[g].max() <= 1e-4


# ------------------------------------------------------------- wide pixels
@pytest.mark.parametrize("case", pc.WIDE)
def test_wide_pixel_parity(case):
    """p*q > 64 (one 4-wave workgroup per pixel): p=5, q=24, n=256 (the
    mixed-precision workload's shape) and p=6, q=16, r_a=2 (two stacked
    3-channel passes)."""
    kstap = _kstap()
    spec, seed, base, prec = pc.wide_case(case)
    sc = scenegen.make_scene(spec, seed=seed)
    plan = kstap.Plan(**base, precision=prec)
    note(f"wide {case}")
    Tg, Dg, xd = run_frame(plan, sc.x)
    ref, out = frame_oracle(sc.x, oracle.OracleConfig(**base))
    check_parity(Tg.ravel(), Dg.ravel(), ref, plan.tau, base["r_a"], base["r_b"], "wide " + case)
    pix = out["pixels"][::7]
    pr = kstap.probe(plan, xd, pix)
    torch.cuda.synchronize()
    sel = np.arange(0, len(out["pixels"]), 7)
    UB = pr["U_B"].cpu().numpy().astype(np.complex128)
    dB = np.abs(UB @ np.conj(np.swapaxes(UB, 1, 2)) - out["U_B"][sel] @ np.conj(np.swapaxes(out["U_B"][sel], 1, 2))).max()
    UA = pr["U_A"].cpu().numpy().astype(np.complex128)
    dA = np.abs(UA @ np.conj(np.swapaxes(UA, 1, 2)) - out["U_A"][sel] @ np.conj(np.swapaxes(out["U_A"][sel], 1, 2))).max()
    # the frame pass updates most covariances from the previous pixel's, the
    # probe sums every pixel's from scratch: they differ by summation order
    eP = rel_err(pr["T"].cpu().numpy(), Tg[pix[:, 0], pix[:, 1]]).max()
    note(f"[wide {case}] probe projector distance A {dA:.2e} B {dB:.2e}, probe vs frame T {eP:.2e}")
    assert eP <= 2e-5
    assert dA <= 1e-4 and dB <= 1e-4
