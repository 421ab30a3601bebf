"""Pins of the variant and multipass oracle (`oracle/variants.py`) against
what the paper and the mathematics fix: projector identities of Eqs. (24) and
(25), brute-force maximisation over the spatial steering (Sec. 6.3), the
closed form of the Kron-STAP statistic from the core oracle (an independent
code path), a closed form of the classical statistic derived by hand, the
Gamma null laws, NumPy's FFT for the single-antenna image of a DFT bank, and
the exact subspace recovery of the K-pass model of Sec. 3.
"""
import numpy as np
import pytest
import scipy.stats

import oracle
from oracle import variants as V
import scenegen


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def rand_basis(rng, m, r):
    Q, _ = np.linalg.qr(crandn(rng, m, r))
    return Q[:, :r]


def proj(U):
    return U @ U.conj().T


# ------------------------------------------------------------ bank (V2)
@pytest.mark.parametrize("q,M", [(8, 8), (16, 16), (12, 5)])
def test_doppler_bank_is_unit_modulus_dft(q, M):
    """Bin m is exp(2 pi j m k / M): unit modulus, bin 0 all ones, and for
    M = q the bins are the orthogonal DFT basis (b_m^H b_m' = q delta)."""
    b = V.doppler_bank(q, M)
    assert b.shape == (M, q)
    np.testing.assert_allclose(np.abs(b), 1.0, atol=1e-15)
    np.testing.assert_allclose(b[0], 1.0, atol=1e-15)
    k = np.arange(q)
    for m in range(M):
        np.testing.assert_allclose(b[m], np.exp(2j * np.pi * m * k / M), atol=1e-12)
    if M == q:
        np.testing.assert_allclose(b.conj() @ b.T, q * np.eye(q), atol=1e-12)


# --------------------------------------------- filters (Eqs. (24), (25))
@pytest.mark.parametrize("kind", ["kron", "classical"])
@pytest.mark.parametrize("p,q,ra,rb", [(3, 4, 1, 2), (2, 5, 1, 3), (4, 3, 2, 1), (3, 4, 1, 0)])
def test_filters_are_orthogonal_projectors(kind, p, q, ra, rb):
    """Both filters are Hermitian idempotent; Eq. (25) has rank
    (p - r_a)(q - r_b) and annihilates U_A (x) anything and anything (x) U_B;
    Eq. (24) has rank pq - r_a r_b and annihilates exactly U_A (x) U_B."""
    rng = np.random.default_rng(p * 100 + q * 10 + ra + rb)
    UA, UB = rand_basis(rng, p, ra), rand_basis(rng, q, rb)
    F = V.filter_matrix(UA[None], UB[None], kind)[0]
    np.testing.assert_allclose(F, F.conj().T, atol=1e-14)
    np.testing.assert_allclose(F @ F, F, atol=1e-13)
    rank = (p - ra) * (q - rb) if kind == "kron" else p * q - ra * rb
    assert np.real(np.trace(F)) == pytest.approx(rank, abs=1e-12)
    if rb > 0:
        np.testing.assert_allclose(F @ np.kron(UA, UB), 0.0, atol=1e-13)
    if kind == "kron":
        np.testing.assert_allclose(F @ np.kron(UA, crandn(rng, q, 1)), 0.0, atol=1e-13)
        if rb > 0:
            np.testing.assert_allclose(F @ np.kron(crandn(rng, p, 1), UB), 0.0, atol=1e-13)
    else:
        # vectors orthogonal to U_A (x) U_B pass unchanged
        v = crandn(rng, p * q)
        v -= proj(np.kron(UA, UB)) @ v
        np.testing.assert_allclose(F @ v, v, atol=1e-13)


# --------------------------------------------- statistic (V1, Sec. 6.3)
def _direct(F, x, h, b):
    d = np.kron(h, b)
    return abs(np.vdot(d, F @ x)) ** 2 / np.real(np.vdot(d, F @ d))


@pytest.mark.parametrize("kind", ["kron", "classical"])
def test_glrt_is_the_maximum_over_spatial_steerings(kind):
    """u^H G^+ u is attained at h = G^+ u (evaluated with the direct ratio
    |d^H F x|^2 / d^H F d on d = h (x) b) and exceeded by none of 2 000
    random steerings."""
    rng = np.random.default_rng(7 if kind == "kron" else 8)
    p, q = 3, 6
    UA, UB = rand_basis(rng, p, 1), rand_basis(rng, q, 2)
    F = V.filter_matrix(UA[None], UB[None], kind)[0]
    b = np.exp(0.7j * np.arange(q))
    for trial in range(4):
        X = crandn(rng, p, q)
        T, u = V.glrt_explicit(F[None], X[None], b)
        E = V.steering_matrix(p, b)
        G = E.conj().T @ F @ E
        hstar = np.linalg.pinv(G, rcond=1e-10) @ u[0]
        assert _direct(F, X.reshape(-1), hstar, b) == pytest.approx(T[0], rel=1e-10)
        hs = crandn(rng, 2000, p)
        x = X.reshape(-1)
        vals = [_direct(F, x, h, b) for h in hs]
        assert max(vals) <= T[0] * (1 + 1e-10)
        assert max(vals) >= 0.9 * T[0]


@pytest.mark.parametrize("mode", ["glrt", "fixed"])
def test_kron_filter_matches_the_core_closed_form(mode):
    """For the Kron-STAP filter the explicit evaluation equals the core
    oracle's closed form ||F_A X conj(F_B b)||^2 / (b^H F_B b) (and its
    fixed-h form), which is computed by different code."""
    rng = np.random.default_rng(21)
    p, q, N = 4, 6, 12
    UA = np.stack([rand_basis(rng, p, 2) for _ in range(N)])
    UB = np.stack([rand_basis(rng, q, 3) for _ in range(N)])
    X = crandn(rng, N, p, q)
    b = np.exp(0.4j * np.arange(q)) * (1 + 0.1 * np.arange(q))
    h = None if mode == "glrt" else crandn(rng, p)
    T_ex, _ = V.glrt_explicit(V.filter_matrix(UA, UB, "kron"), X, b, h)
    T_cf = oracle.kron_stap_statistic(X, UA, UB, b, h)
    np.testing.assert_allclose(T_ex, T_cf, rtol=1e-10)


def test_classical_filter_matches_a_hand_derived_closed_form():
    """With F = I - P_A (x) P_B, G = ||b||^2 F_A + (b^H F_B b) P_A, so
    max_h = ||F_A X b*||^2 / ||b||^2 + ||P_A X conj(F_B b)||^2 / (b^H F_B b)."""
    rng = np.random.default_rng(22)
    p, q, N = 3, 8, 10
    for ra, rb in ((1, 3), (2, 2), (1, 0)):
        UA = np.stack([rand_basis(rng, p, ra) for _ in range(N)])
        UB = np.stack([rand_basis(rng, q, rb) for _ in range(N)])
        X = crandn(rng, N, p, q)
        b = np.exp(1j * rng.uniform(0, 2 * np.pi, q))
        T_ex, _ = V.glrt_explicit(V.filter_matrix(UA, UB, "classical"), X, b)
        for i in range(N):
            PA, PB = proj(UA[i]), proj(UB[i])
            FA, FB = np.eye(p) - PA, np.eye(q) - PB
            t1 = np.linalg.norm(FA @ X[i] @ b.conj()) ** 2 / np.vdot(b, b).real
            g = FB @ b
            t2 = np.linalg.norm(PA @ X[i] @ g.conj()) ** 2 / np.vdot(b, g).real
            assert T_ex[i] == pytest.approx(t1 + t2, rel=1e-10)


def test_classical_statistic_null_law_is_gamma_p():
    """Reading V4: white noise, exact subspaces -> T ~ Gamma(p, 1) (KS), and
    the default threshold is SciPy's Gamma(p) quantile."""
    rng = np.random.default_rng(23)
    p, q, N = 3, 8, 6000
    UA, UB = rand_basis(rng, p, 1), rand_basis(rng, q, 3)
    F = V.filter_matrix(UA[None], UB[None], "classical")
    X = crandn(rng, N, p, q)
    T, _ = V.glrt_explicit(np.broadcast_to(F, (N,) + F.shape[1:]), X, np.ones(q))
    assert scipy.stats.kstest(T, scipy.stats.gamma(p).cdf).pvalue > 1e-3
    cfg = V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3, filter="classical")
    assert cfg.threshold() == pytest.approx(scipy.stats.gamma(3).isf(1e-4), rel=1e-9)
    cfg = V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3)
    assert cfg.threshold() == pytest.approx(scipy.stats.gamma(2).isf(1e-4), rel=1e-9)


def test_fixed_h_is_below_the_maximum_and_equals_the_direct_ratio():
    rng = np.random.default_rng(24)
    p, q = 3, 6
    UA, UB = rand_basis(rng, p, 1), rand_basis(rng, q, 2)
    b = np.ones(q)
    for kind in ("kron", "classical"):
        F = V.filter_matrix(UA[None], UB[None], kind)
        X = crandn(rng, 1, p, q)
        h = crandn(rng, p)
        Tf, _ = V.glrt_explicit(F, X, b, h)
        Tg, _ = V.glrt_explicit(F, X, b)
        assert Tf[0] == pytest.approx(_direct(F[0], X[0].reshape(-1), h, b), rel=1e-10)
        assert Tf[0] <= Tg[0] * (1 + 1e-12)


# ------------------------------------------------ enhancement image (V3)
def test_sar_intensity_of_a_dft_bank_is_numpy_fft():
    """For the M = q bank, channel 0's matched-filter intensity at bin m is
    |FFT(X[0])[m]|^2 / q."""
    rng = np.random.default_rng(25)
    q = 16
    X = crandn(rng, 5, 3, q)
    bank = V.doppler_bank(q, q)
    f = np.fft.fft(X[:, 0, :], axis=1)
    for m in range(q):
        np.testing.assert_allclose(V.sar_intensity(X, bank[m]), np.abs(f[:, m]) ** 2 / q, rtol=1e-12)


# ---------------------------------------------------- whole-pixel checks
def _small_scene(seed=31, **kw):
    spec = scenegen.SceneSpec(p=3, q=8, H=22, W=22, r_a=1, r_b=3, n_targets=3, snr_db=12.0, **kw)
    return scenegen.make_scene(spec, seed=seed)


def test_variant_pixels_reduce_to_the_core_oracle():
    """filter='kron', no bank, one pass: T, D, subspaces equal the core
    oracle's; the enhancement is T / I_SAR with I_SAR from channel 0."""
    sc = _small_scene()
    cfg = V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3)
    pix = scenegen.random_pixels(22, 22, 60, 3)
    a = V.variant_pixels(sc.x, pix, cfg)
    b = oracle.kron_stap_pixels(sc.x, pix, oracle.OracleConfig(p=3, q=8, n=64, r_a=1, r_b=3))
    np.testing.assert_allclose(a["T"], b["T"], rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(a["D"], b["D"])
    v = a["valid"]
    Xt = oracle.snapshots(sc.x, pix[v, 0], pix[v, 1])
    isar = np.abs(Xt[:, 0, :].sum(1)) ** 2 / 8
    np.testing.assert_allclose(a["E"][v], a["T"][v] / isar, rtol=1e-12)
    assert np.all(a["bin"] == 0)


def test_bank_is_the_maximum_of_single_steering_runs():
    """The bank statistic is the maximum over bins of single-steering runs
    with b_steer = b_m, the bin its first maximiser; a one-bin bank is the
    all-ones steering."""
    sc = _small_scene(seed=32)
    pix = scenegen.random_pixels(22, 22, 40, 4)
    cfg = V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3, nbank=6)
    a = V.variant_pixels(sc.x, pix, cfg)
    singles = np.stack([V.variant_pixels(sc.x, pix, V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3, b_steer=bm))["T"]
                        for bm in V.doppler_bank(8, 6)], 1)
    np.testing.assert_allclose(a["T"], singles.max(1), rtol=1e-12)
    np.testing.assert_array_equal(a["bin"][a["valid"]], np.argmax(singles, 1)[a["valid"]])
    one = V.variant_pixels(sc.x, pix, V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3, nbank=1))
    ref = V.variant_pixels(sc.x, pix, V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3))
    np.testing.assert_allclose(one["T"], ref["T"], rtol=1e-12)


def test_bank_enhancement_divides_by_the_fft_image_at_the_chosen_bin():
    """With an M = q bank the enhancement is T over channel 0's SAR image at
    the chosen bin, |FFT(X[0])[bin]|^2 / q (Sec. 6.3)."""
    sc = _small_scene(seed=34)
    pix = scenegen.random_pixels(22, 22, 40, 8)
    o = V.variant_pixels(sc.x, pix, V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3, nbank=8))
    v = o["valid"]
    Xt = oracle.snapshots(sc.x, pix[v, 0], pix[v, 1])
    f = np.fft.fft(Xt[:, 0, :], axis=1)
    isar = np.abs(f[np.arange(f.shape[0]), o["bin"][v]]) ** 2 / 8
    np.testing.assert_allclose(o["E"][v], o["T"][v] / isar, rtol=1e-10)
    assert len(set(o["bin"][v].tolist())) > 1


def test_classical_on_pixels_uses_the_gamma_p_threshold():
    """A classical-filter run thresholds at the Gamma(p) quantile (V4) and,
    on the same estimates, its statistic is the explicit GLRT of Eq. (24)."""
    sc = _small_scene(seed=33)
    pix = scenegen.random_pixels(22, 22, 40, 5)
    tc = V.variant_pixels(sc.x, pix, V.VariantConfig(p=3, q=8, n=64, r_a=1, r_b=3, filter="classical"))
    assert tc["tau"] == pytest.approx(scipy.stats.gamma(3).isf(1e-4), rel=1e-9)
    v = tc["valid"]
    np.testing.assert_array_equal(tc["D"][v], (tc["T"][v] > tc["tau"]).astype(np.uint8))
    Xt = oracle.snapshots(sc.x, pix[v, 0], pix[v, 1])
    F = V.filter_matrix(tc["U_A"][v], tc["U_B"][v], "classical")
    for i in range(int(v.sum())):
        x = Xt[i].reshape(-1)
        E = V.steering_matrix(3, np.ones(8))
        G = E.conj().T @ F[i] @ E
        u = E.conj().T @ F[i] @ x
        assert tc["T"][v][i] == pytest.approx(np.real(np.vdot(u, np.linalg.solve(G, u))), rel=1e-9)


# --------------------------------------------------- multipass (Sec. 3)
MP = scenegen.MultipassSpec(passes=2, p=3, q=6, H=20, W=20, r_b=2, coherence=0.8, n_targets=2)


def test_multipass_model_has_rank_k_space_factor():
    """Sec. 3: A_tilde is Kp x Kp of rank K, its range spanned by the per-pass
    spatial factors placed in their pass's block."""
    rng = np.random.Generator(np.random.PCG64(5))
    A, B, U = scenegen.multipass_factors(MP, rng)
    lam = np.linalg.eigvalsh(A)[::-1]
    assert lam[1] > 1e-6 * lam[0] and abs(lam[2]) < 1e-12 * lam[0]
    lam_b = np.linalg.eigvalsh(B)[::-1]
    assert lam_b[MP.r_b - 1] > 0 and abs(lam_b[MP.r_b]) < 1e-10 * lam_b[0]
    np.testing.assert_allclose(proj(np.linalg.eigh(A)[1][:, ::-1][:, :2]), proj(U), atol=1e-12)
    for k in range(2):
        assert np.count_nonzero(np.abs(U[:, k]) > 0) == MP.p


def test_multipass_exact_model_is_recovered():
    """Sec. 3 + Algorithm 2: on S = A_tilde (x) B the LR-Kron fit with
    r_a = K reproduces S (eta = 0) and U_A spans the K-pass subspace; with
    white noise added the subspaces are still exact (as pin P4)."""
    rng = np.random.Generator(np.random.PCG64(6))
    A, B, U = scenegen.multipass_factors(MP, rng)
    P, q = 2 * MP.p, MP.q
    S = np.kron(A, B)
    est = oracle.lr_kron(oracle.rearrange(S, P, q), P, q, 2, MP.r_b)
    assert est["eta"] < 1e-12
    np.testing.assert_allclose(np.kron(est["A"], est["B"]), S, atol=1e-9 * np.abs(S).max())
    np.testing.assert_allclose(proj(est["U_A"]), proj(U), atol=1e-10)
    est = oracle.lr_kron(oracle.rearrange(0.3 * S + np.eye(P * q), P, q), P, q, 2, MP.r_b)
    np.testing.assert_allclose(proj(est["U_A"]), proj(U), atol=1e-10)
    ub = np.linalg.eigh(B)[1][:, ::-1][:, :MP.r_b]
    np.testing.assert_allclose(proj(est["U_B"]), proj(ub), atol=1e-10)


def _mp_scene():
    return scenegen.make_multipass_scene(MP, seed=41)


def test_pass_images_sum_to_the_joint_statistic():
    """||u||^2 splits over the passes' channels: sum_k T_k = T (reading V5)."""
    sc = _mp_scene()
    cfg = V.VariantConfig(p=6, q=6, n=64, r_a=2, r_b=2, passes=2)
    pix = scenegen.random_pixels(20, 20, 50, 6)
    o = V.variant_pixels(sc.x, pix, cfg)
    v = o["valid"]
    np.testing.assert_allclose(o["T_pass"][v].sum(1), o["T"][v], rtol=1e-10)
    np.testing.assert_allclose(o["C"][v, 0], np.sqrt(o["T_pass"][v, 1]) - np.sqrt(o["T_pass"][v, 0]), rtol=1e-12)


def test_swapping_passes_swaps_images_and_negates_change():
    sc = _mp_scene()
    cfg = V.VariantConfig(p=6, q=6, n=64, r_a=2, r_b=2, passes=2)
    pix = scenegen.random_pixels(20, 20, 40, 7)
    a = V.variant_pixels(sc.x, pix, cfg)
    xs = np.ascontiguousarray(np.concatenate([sc.x[3:], sc.x[:3]], 0))
    b = V.variant_pixels(xs, pix, cfg)
    v = a["valid"]
    np.testing.assert_allclose(b["T_pass"][v][:, ::-1], a["T_pass"][v], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(b["C"][v], -a["C"][v], rtol=1e-6, atol=1e-7)


def test_pass_images_vanish_on_in_subspace_clutter():
    """A test snapshot whose columns lie in span(U_A) gives T_k = 0 for every
    pass (Eq. (25) projects the spatial subspace away)."""
    rng = np.random.default_rng(43)
    P, q, N = 6, 6, 5
    UA = np.stack([rand_basis(rng, P, 2) for _ in range(N)])
    UB = np.stack([rand_basis(rng, q, 2) for _ in range(N)])
    X = np.matmul(UA, crandn(rng, N, 2, q))
    _, u = V.glrt_explicit(V.filter_matrix(UA, UB, "kron"), X, np.ones(q))
    np.testing.assert_allclose(u, 0.0, atol=1e-12)
