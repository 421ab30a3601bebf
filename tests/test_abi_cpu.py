"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/kstap.h, validates configurations, and its
stencil / threshold / valid-region logic agrees with the oracle's independent
implementation."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1604_03622_amd as kstap


def test_library_exports_every_declared_symbol():
    L = kstap.lib()
    names = kstap.exported_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert "gfx950" in kstap.version()


@pytest.mark.parametrize("n", [64, 128, 200, 256, 17])
def test_default_stencil_matches_oracle(n):
    plan = kstap.Plan(p=3, q=16, n=n, r_a=1, r_b=4)
    np.testing.assert_array_equal(plan.stencil, oracle.default_stencil(n))
    assert plan.window == oracle.stencil_window(n)


def test_explicit_stencil_and_valid_region():
    st = oracle.default_stencil(40, window=12, guard=5)
    plan = kstap.Plan(p=3, q=8, n=40, stencil=st)
    np.testing.assert_array_equal(plan.stencil, st)
    for H, W in ((64, 64), (20, 37), (5, 5)):
        assert plan.valid_region(H, W) == oracle.valid_region(H, W, st)


@pytest.mark.parametrize("p,ra,pfa", [(3, 1, 1e-4), (4, 1, 1e-4), (3, 2, 1e-3), (6, 1, 1e-6), (4, 2, 1e-5)])
def test_threshold_matches_gamma_quantile(p, ra, pfa):
    plan = kstap.Plan(p=p, q=8, n=64, r_a=ra, r_b=3, pfa=pfa)
    assert plan.tau == pytest.approx(oracle.gamma_upper_quantile(p - ra, pfa), rel=1e-12)
    assert kstap.Plan(p=3, q=8, n=64, tau=7.5).tau == 7.5


@pytest.mark.parametrize("kw,status", [
    (dict(p=0), 1), (dict(p=9), 1), (dict(q=1), 1), (dict(q=33), 1), (dict(n=0), 1), (dict(n=257), 1),
    (dict(r_a=0), 1), (dict(r_a=4), 1), (dict(r_b=9), 1), (dict(min_iter=0), 1), (dict(min_iter=5, max_iter=4), 1),
    (dict(guard=2), 1), (dict(window=11), 1), (dict(window=10, n=100), 1), (dict(pfa=0.0), 1),
    (dict(stat_mode="fixed"), 1), (dict(stencil=[[0, 0]] * 64), 1), (dict(stencil=[[1, 2]] * 64), 1),
    (dict(p=7, q=16), 2), (dict(p=1), 2),
])
def test_plan_validation_errors(kw, status):
    args = dict(p=3, q=8, n=64, r_a=1, r_b=3)
    args.update(kw)
    with pytest.raises(kstap.StapError) as ei:
        kstap.Plan(**args)
    assert ei.value.status == status
    assert kstap.lib().stap_last_error().decode() != ""


def test_run_rejects_bad_arguments_without_touching_a_device():
    plan = kstap.Plan(p=3, q=8, n=64)
    L = kstap.lib()
    assert L.stap_run(plan.handle, None, 64, 64, ctypes.c_void_p(16), None, None) == 1
    assert L.stap_run(plan.handle, ctypes.c_void_p(16), 0, 64, ctypes.c_void_p(16), None, None) == 1
    assert L.stap_run(plan.handle, ctypes.c_void_p(16), 64, 64, None, None, None) == 1
    assert L.stap_run(plan.handle, ctypes.c_void_p(16), 40000, 40000, ctypes.c_void_p(16), None, None) == 1
    assert L.stap_run(None, ctypes.c_void_p(16), 64, 64, ctypes.c_void_p(16), None, None) == 1
    out = kstap.StapProbeOut(None, None, None, None, None)
    assert L.stap_probe(plan.handle, ctypes.c_void_p(16), 64, 64, ctypes.c_void_p(16), 3, ctypes.byref(out), None) == 1
    assert L.stap_probe(plan.handle, ctypes.c_void_p(16), 64, 64, None, -1, None, None) == 1


def test_batch_rejects_bad_arguments_without_a_device():
    L = kstap.lib()
    h = ctypes.c_void_p()
    assert L.stap_batch_create(None, 0, 0, ctypes.byref(h)) == 1
    arr = (kstap.StapTile * 1)()
    arr[0] = kstap.StapTile(None, 16, 8, 8, 16, None)
    assert L.stap_batch_create(arr, 1, 0, ctypes.byref(h)) == 1
    assert L.stap_batch_create(arr, 1, -3, ctypes.byref(h)) == 1
    assert L.stap_batch_launch(None, None) == 1
    assert L.stap_batch_tune(None, None, None, None, None) == 1
    assert L.stap_batch_destroy(None) == 0
    assert L.stap_run_batch(None, 0, None) == 1


def test_server_rejects_bad_arguments_without_a_device():
    L = kstap.lib()
    h = ctypes.c_void_p()
    assert L.stap_server_create(1 << 10, 4, 0, ctypes.byref(h)) == 1
    assert L.stap_server_create(1 << 30, 0, 0, ctypes.byref(h)) == 1
    assert L.stap_server_create(1 << 30, 4, -1, ctypes.byref(h)) == 1
    assert L.stap_server_create(1 << 30, 4, 0, None) == 1
    t = ctypes.c_uint64()
    assert L.stap_server_submit(None, None, None, 8, 8, 0, None, None, None, ctypes.byref(t)) == 1
    assert L.stap_server_wait(None, 1, 0, None) == 1
    assert L.stap_server_stats(None, None, None, None, None) == 1
    assert L.stap_server_destroy(None) == 0


# --------------------------------------------- sliding-window bookkeeping
# The kernels update a pixel's covariance from the previous pixel's when the
# order says it is a one-pixel move; these checks pin the order and the
# entering / leaving lists on the host, against set algebra on the stencil.
MOVE_D = {0: (0, 1), 1: (0, -1), 2: (1, 0)}


@pytest.mark.parametrize("p,q,H,W", [(3, 16, 64, 64), (3, 8, 37, 53), (3, 16, 130, 70), (5, 24, 70, 130),
                                     (6, 16, 9, 5)])
def test_order_visits_every_pixel_once_and_moves_are_neighbours(p, q, H, W):
    plan = kstap.Plan(p=p, q=q, n=64, r_a=1, r_b=3)
    pix, mv = plan.order(H, W)
    inside = pix[:, 0] >= 0
    seen = pix[inside]
    assert len(seen) == H * W
    assert len({(int(r), int(c)) for r, c in seen}) == H * W
    chain = 64 if p * q > 64 else 16
    assert np.all(mv[::chain] == -1)
    for i in np.nonzero(mv >= 0)[0]:
        if not (inside[i] and inside[i - 1]):
            continue   # the kernels break the chain at the frame's edge
        dr, dc = MOVE_D[int(mv[i])]
        assert tuple(pix[i] - pix[i - 1]) == (dr, dc), (i, pix[i - 1], pix[i], mv[i])
    # chains are long: only a few positions start one
    assert np.mean(mv == -1) <= (1.5 / chain if chain == 16 else 2.5 / chain)


@pytest.mark.parametrize("n", [64, 128, 200, 256])
def test_move_lists_are_the_stencil_set_differences(n):
    plan = kstap.Plan(p=3, q=16, n=n, r_a=1, r_b=4)
    st = {tuple(map(int, o)) for o in oracle.default_stencil(n)}
    for mv, (dr, dc) in MOVE_D.items():
        add, rem = plan.moves(mv)
        add = {tuple(map(int, o)) for o in add}
        rem = {tuple(map(int, o)) for o in rem}
        prev = {(a - dr, b - dc) for a, b in st}   # previous pixel's stencil, seen from the new pixel
        assert add == st - prev and rem == prev - st
        assert (prev - rem) | add == st
