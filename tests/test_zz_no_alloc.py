"""stap_run_noalloc (the whole-frame pass that allocates nothing: the mixed
path's split planes live in a static per-device work area) against stap_run,
through the C ABI, on two calls in a row with the second frame smaller, so the
second call reuses the work area the first one filled."""
import numpy as np
import pytest

import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kstap():
    import paper_1604_03622_amd as kstap
    return kstap


def _frame(spec_kw, seed):
    sc = scenegen.make_scene(scenegen.SceneSpec(**spec_kw), seed=seed)
    return torch.from_numpy(sc.x).to("cuda:0")


def _both(kstap, plan, x):
    H, W = x.shape[1], x.shape[2]
    T1, D1 = kstap.run(plan, x)
    T2 = torch.full((H, W), -1.0, device=x.device)
    D2 = torch.full((H, W), 7, dtype=torch.uint8, device=x.device)
    kstap.run_noalloc(plan, x, T2, D2)
    torch.cuda.synchronize()
    return T1.cpu().numpy(), D1.cpu().numpy(), T2.cpu().numpy(), D2.cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp32_f64"])
def test_noalloc_equals_run_twice_shrinking(prec):
    kstap = _kstap()
    base = dict(p=3, q=16, n=200, r_a=1, r_b=4)
    plan = kstap.Plan(**base, precision=prec)
    for i, (H, W) in enumerate(((96, 100), (41, 57))):
        print(f"noalloc {prec} call {i}: {H}x{W}", flush=True)
        x = _frame(dict(p=3, q=16, H=H, W=W, r_a=1, r_b=4, n_targets=4, snr_db=(0.0, 15.0), block=32),
                   scenegen.BASE_SEED + 600 + i)
        T1, D1, T2, D2 = _both(kstap, plan, x)
        # same kernel and the same plane contents: the results are bitwise equal
        assert np.array_equal(T1, T2), f"call {i}: T differs, max {np.abs(T1 - T2).max()}"
        assert np.array_equal(D1, D2)
        r0, r1, c0, c1 = plan.valid_region(H, W)
        inner = np.zeros((H, W), bool)
        inner[r0:r1, c0:c1] = True
        assert (T2[inner] > 0).all() and (T2[~inner] == 0).all()


def test_noalloc_wide_and_small_class():
    """A wide-pixel plan (no planes) and a q = 8 mixed plan after the larger
    calls above have left their contents in the work area."""
    kstap = _kstap()
    for base, prec, H, W in ((dict(p=5, q=24, n=256, r_a=1, r_b=4), "bf16x3", 40, 44),
                             (dict(p=3, q=8, n=64, r_a=1, r_b=3), "bf16x3", 33, 30)):
        print(f"noalloc {base} {prec} {H}x{W}", flush=True)
        plan = kstap.Plan(**base, precision=prec)
        x = _frame(dict(p=base["p"], q=base["q"], H=H, W=W, r_a=1, r_b=base["r_b"], n_targets=2),
                   scenegen.BASE_SEED + 610 + base["q"])
        T1, D1, T2, D2 = _both(kstap, plan, x)
        assert np.array_equal(T1, T2) and np.array_equal(D1, D2)


def test_noalloc_refuses_oversize_frame():
    """A mixed-path frame whose planes exceed the work area is refused on the
    host before anything is enqueued; T is left untouched."""
    kstap = _kstap()
    plan = kstap.Plan(p=3, q=16, n=200, r_a=1, r_b=4, precision="bf16x3")
    H = W = 600   # 3 * 600 * 600 * 16 samples * 8 bytes > 128 MiB
    assert 3 * H * W * 16 * 8 > kstap.NOALLOC_MAX_BYTES
    x = torch.zeros((3, H, W, 16), dtype=torch.complex64, device="cuda:0")
    T = torch.full((H, W), -1.0, device=x.device)
    with pytest.raises(kstap.StapError) as ei:
        kstap.run_noalloc(plan, x, T)
    assert ei.value.status == 1
    torch.cuda.synchronize()
    assert bool((T == -1.0).all())
