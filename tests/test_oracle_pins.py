"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the property it pins and the passage it comes from.  None of
them re-types the oracle's own formula: they use closed forms (Kronecker
identities), library routines for special cases (SVD, SciPy's Gamma law,
mpmath's high-precision eigensolver), brute force, and invariants.
"""
import numpy as np
import pytest
import scipy.stats

import oracle
from oracle.kron_stap import _unvec, _vec
import scenegen


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


def rand_psd(rng, m, r):
    g = crandn(rng, m, r)
    return g @ g.conj().T


def proj(U):
    return U @ U.conj().T


def range_proj(M, r):
    lam, V = np.linalg.eigh((M + M.conj().T) / 2)
    U = V[:, ::-1][:, :r]
    return proj(U)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("p,q", [(2, 3), (3, 8), (4, 5), (5, 2)])
def test_p1_rearrangement_of_kronecker_is_rank_one(p, q):
    """Alg. 1 / Eq. (16): R(A (x) B) = vec(A) vec(B)^T, and R permutes S's entries."""
    rng = np.random.default_rng(1 + p * 10 + q)
    A, B = crandn(rng, p, p), crandn(rng, q, q)
    R = oracle.rearrange(np.kron(A, B), p, q)
    assert R.shape == (p * p, q * q)
    np.testing.assert_array_equal(R, np.outer(_vec(A), _vec(B)))
    S = crandn(rng, p * q, p * q)
    R = oracle.rearrange(S, p, q)
    assert np.linalg.norm(R) == pytest.approx(np.linalg.norm(S), rel=1e-15)
    np.testing.assert_array_equal(np.sort_complex(R.ravel()), np.sort_complex(S.ravel()))
    np.testing.assert_array_equal(R, oracle.rearrange_direct(S, p, q))


def test_p1_index_grid_is_a_bijection():
    """Alg. 1 with reading R4 addresses every entry of vec(S) exactly once."""
    p, q = 3, 4
    S = np.arange((p * q) ** 2, dtype=float).reshape(p * q, p * q) + 1.0
    R = oracle.rearrange(S, p, q)
    assert sorted(R.ravel().tolist()) == sorted(S.ravel().tolist())


# ---------------------------------------------------------------- P2
def test_p2_initialiser_equals_block_sum_form():
    """Eq. (18) a_0 = R 1 / q^2 equals Eq. (19) (1/q^2)(I (x) 1)^T S (I (x) 1)."""
    rng = np.random.default_rng(2)
    p, q, n = 3, 6, 20
    X = crandn(rng, p * q, n)
    S = X @ X.conj().T / n
    R = oracle.rearrange(S, p, q)
    a0 = R @ np.ones(q * q) / q ** 2
    E = np.kron(np.eye(p), np.ones((q, 1)))
    A0 = E.T @ S @ E / q ** 2
    np.testing.assert_allclose(_unvec(a0, p), A0, rtol=0, atol=1e-14 * np.abs(A0).max())
    assert np.linalg.eigvalsh(A0).min() >= -1e-12 * np.abs(A0).max()


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("p,q,ra,rb", [(3, 8, 1, 3), (3, 16, 1, 4), (5, 6, 2, 2)])
def test_p3_exact_kronecker_is_recovered(p, q, ra, rb):
    """S = A (x) B with rank(A) <= r_a, rank(B) <= r_b: A-hat (x) B-hat = S, eta = 0."""
    rng = np.random.default_rng(3 + p + q)
    A, B = rand_psd(rng, p, ra), rand_psd(rng, q, rb)
    S = np.kron(A, B)
    out = oracle.lr_kron(oracle.rearrange(S, p, q), p, q, ra, rb, eps=1e-14, min_iter=1, max_iter=1)
    Bhat, _, _ = oracle.eig_truncate(out["B"], rb)
    np.testing.assert_allclose(np.kron(out["A"], Bhat), S, atol=1e-12 * np.abs(S).max())
    assert out["eta"] < 1e-13
    assert out["iters"] == 1


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("ra", [1, 2])
def test_p4_population_covariance_plus_noise_gives_exact_subspaces(ra):
    """S = c A (x) B + sigma^2 I: U_A spans range(A), U_B spans range(B) exactly
    (R(I) = vec(I_p) vec(I_q)^T keeps every iterate in span{A, I}, span{B, I})."""
    rng = np.random.default_rng(40 + ra)
    p, q, rb = 4, 10, 3
    A, B = rand_psd(rng, p, ra), rand_psd(rng, q, rb)
    S = 50.0 * np.kron(A, B) + 0.7 * np.eye(p * q)
    out = oracle.lr_kron(oracle.rearrange(S, p, q), p, q, ra, rb, eps=1e-15, max_iter=30)
    np.testing.assert_allclose(proj(out["U_A"]), range_proj(A, ra), atol=1e-12)
    np.testing.assert_allclose(proj(out["U_B"]), range_proj(B, rb), atol=1e-12)
    # the conjugate subspace is a different subspace: the test can tell them apart
    assert np.abs(proj(out["U_A"]) - range_proj(A.conj(), ra)).max() > 1e-3


# ---------------------------------------------------------------- P5
def test_p5_full_ranks_give_nearest_kronecker_product():
    """r_a = p, r_b = q: Alg. 2 is power iteration on R; the fit is the leading
    singular pair of R (Van Loan-Pitsianis nearest Kronecker product)."""
    rng = np.random.default_rng(5)
    p, q = 3, 5
    A, B = rand_psd(rng, p, p), rand_psd(rng, q, q)
    X = crandn(rng, p * q, 40)
    S = 4.0 * np.kron(A, B) + X @ X.conj().T / 40
    R = oracle.rearrange(S, p, q)
    out = oracle.lr_kron(R, p, q, p, q, eps=0.0, max_iter=300)
    fit = np.outer(_vec(out["A"]), _vec(out["B"]))
    u, s, vh = np.linalg.svd(R)
    best = s[0] * np.outer(u[:, 0], vh[0])
    np.testing.assert_allclose(fit, best, atol=1e-10 * s[0])


# ---------------------------------------------------------------- P6
def test_p6_factors_are_psd():
    """Sec. 4: the PSD initialisation makes A-hat (x) B-hat PSD Hermitian."""
    rng = np.random.default_rng(6)
    p, q, n = 3, 8, 12
    for _ in range(20):
        X = crandn(rng, p * q, n)
        S = X @ X.conj().T / n
        out = oracle.lr_kron(oracle.rearrange(S, p, q), p, q, 2, 3)
        for M in (out["A"], out["B"]):
            np.testing.assert_allclose(M, M.conj().T, atol=1e-13 * np.abs(M).max())
            lam = np.linalg.eigvalsh(M)
            assert lam.min() >= -1e-12 * lam.max()


# ---------------------------------------------------------------- P7
def test_p7_projectors_and_factored_statistic():
    """Eq. (25): F_A, F_B, F_A (x) F_B are Hermitian idempotent with traces
    p - r_a, q - r_b, (p - r_a)(q - r_b); the factored statistic equals the
    explicit |d^H F x|^2 / (d^H F d) with d = h (x) b_s (Eqs. (23), (26))."""
    rng = np.random.default_rng(7)
    p, q, ra, rb = 3, 8, 1, 3
    UA = np.linalg.qr(crandn(rng, p, ra))[0]
    UB = np.linalg.qr(crandn(rng, q, rb))[0]
    FA, FB = np.eye(p) - proj(UA), np.eye(q) - proj(UB)
    F = np.kron(FA, FB)
    for M, tr in ((FA, p - ra), (FB, q - rb), (F, (p - ra) * (q - rb))):
        np.testing.assert_allclose(M, M.conj().T, atol=1e-14)
        np.testing.assert_allclose(M @ M, M, atol=1e-13)
        assert np.trace(M).real == pytest.approx(tr, abs=1e-12)
    X = crandn(rng, p, q)
    h, bs = crandn(rng, p), crandn(rng, q)
    d = np.kron(h, bs)
    x = X.reshape(p * q)                       # vec(X^T): x[i*q + j] = X[i, j]
    direct = np.abs(d.conj() @ F @ x) ** 2 / np.real(d.conj() @ F @ d)
    T = oracle.kron_stap_statistic(X, UA, UB, bs, h=h)
    assert T == pytest.approx(direct, rel=1e-12)


# ---------------------------------------------------------------- P8
def test_p8_in_subspace_clutter_gives_zero_statistic():
    """Test snapshots whose rows lie in span(U_B) or columns in span(U_A) are
    cancelled completely by F_A (x) F_B."""
    rng = np.random.default_rng(8)
    p, q, ra, rb = 3, 16, 1, 4
    UA = np.linalg.qr(crandn(rng, p, ra))[0]
    UB = np.linalg.qr(crandn(rng, q, rb))[0]
    bs = np.ones(q)
    X_rows = crandn(rng, p, rb) @ UB.T          # row i of X is (U_B c_i)^T
    X_cols = UA @ crandn(rng, ra, q)            # every column in span(U_A)
    scale = np.abs(X_rows).max() ** 2
    assert oracle.kron_stap_statistic(X_rows, UA, UB, bs) <= 1e-28 * scale
    assert oracle.kron_stap_statistic(X_cols, UA, UB, bs) <= 1e-28 * np.abs(X_cols).max() ** 2
    # a snapshot outside both subspaces is not cancelled
    assert oracle.kron_stap_statistic(crandn(rng, p, q), UA, UB, bs) > 1e-3


def test_p8_clutter_drawn_from_the_model_is_cancelled():
    """Clutter x = (P (x) Q) w has rows in range(B)^T and columns in range(A):
    with the exact subspaces the statistic of pure clutter is 0."""
    rng = np.random.default_rng(81)
    p, q, ra, rb = 3, 8, 1, 3
    A, B = rand_psd(rng, p, ra), rand_psd(rng, q, rb)
    lamA, VA = np.linalg.eigh(A)
    lamB, VB = np.linalg.eigh(B)
    Pa = (VA * np.sqrt(np.clip(lamA, 0, None))) @ VA.conj().T
    Qb = (VB * np.sqrt(np.clip(lamB, 0, None))) @ VB.conj().T
    Xc = Pa @ crandn(rng, p, q) @ Qb.T
    UA, UB = VA[:, ::-1][:, :ra], VB[:, ::-1][:, :rb]
    T = oracle.kron_stap_statistic(Xc, UA, UB, np.ones(q))
    assert T <= 1e-25 * np.abs(Xc).max() ** 2


# ---------------------------------------------------------------- P9
@pytest.mark.parametrize("k,printed", [(2, 11.756371), (4, 15.913814)])
def test_p9_threshold_matches_gamma_law(k, printed):
    """tau = Gamma(k, 1) upper-tail quantile (the statistic's null law)."""
    tau = oracle.gamma_upper_quantile(k, 1e-4)
    assert tau == pytest.approx(scipy.stats.gamma.isf(1e-4, k), rel=1e-12)
    assert tau == pytest.approx(printed, abs=5e-7)


def test_p9_null_distribution_is_gamma():
    """White-noise test snapshots with fixed subspaces: T ~ Gamma(p - r_a, 1)."""
    rng = np.random.default_rng(9)
    p, q, ra, rb, N = 3, 8, 1, 3, 20000
    UA = np.linalg.qr(crandn(rng, p, ra))[0]
    UB = np.linalg.qr(crandn(rng, q, rb))[0]
    X = crandn(rng, N, p, q)
    T = oracle.kron_stap_statistic(X, np.broadcast_to(UA, (N, p, ra)),
                                   np.broadcast_to(UB, (N, q, rb)), np.ones(q))
    assert scipy.stats.kstest(T, scipy.stats.gamma(p - ra).cdf).pvalue > 1e-3
    assert T.mean() == pytest.approx(p - ra, rel=0.03)


# ---------------------------------------------------------------- P10
def test_p10_glrt_equals_brute_force_maximum_over_h():
    """Sec. 6.3 takes the max over spatial steerings h; the closed form
    ||F_A X conj(F_B b_s)||^2 / (b_s^H F_B b_s) is that maximum of the
    normalised output, attained at h = z."""
    rng = np.random.default_rng(10)
    p, q, ra, rb = 3, 6, 1, 2
    UA = np.linalg.qr(crandn(rng, p, ra))[0]
    UB = np.linalg.qr(crandn(rng, q, rb))[0]
    F = np.kron(np.eye(p) - proj(UA), np.eye(q) - proj(UB))
    X = crandn(rng, p, q)
    bs = crandn(rng, q)
    x = X.reshape(p * q)
    T = oracle.kron_stap_statistic(X, UA, UB, bs)
    H = crandn(rng, 200000, p)
    D = (H[:, :, None] * bs[None, None, :]).reshape(-1, p * q)
    num = np.abs((D.conj() @ F) @ x) ** 2
    den = np.real(np.einsum("ki,ij,kj->k", D.conj(), F, D))
    brute = (num / den).max()
    assert brute <= T * (1 + 1e-12)
    assert brute >= T * (1 - 2e-3)
    # the maximiser: h = F_A X conj(F_B b_s)
    g = (np.eye(q) - proj(UB)) @ bs
    z = (np.eye(p) - proj(UA)) @ X @ g.conj()
    d = np.kron(z, bs)
    assert np.abs(d.conj() @ F @ x) ** 2 / np.real(d.conj() @ F @ d) == pytest.approx(T, rel=1e-12)
    assert oracle.kron_stap_statistic(X, UA, UB, bs, h=z) == pytest.approx(T, rel=1e-12)


# ---------------------------------------------------------------- P11
def test_p11_eigensolver_closed_form_2x2():
    a, d, b = 2.0, -1.0, 1.5 - 0.5j
    M = np.array([[a, b], [np.conj(b), d]])
    lam, U, _ = oracle.top_eigvecs(M, 1)
    disc = np.sqrt(((a - d) / 2) ** 2 + abs(b) ** 2)
    assert lam[0] == pytest.approx((a + d) / 2 + disc, rel=1e-14)
    assert lam[1] == pytest.approx((a + d) / 2 - disc, rel=1e-14)
    v = np.array([b, lam[0] - a])
    v = v / np.linalg.norm(v)
    assert abs(abs(np.vdot(v, U[:, 0])) - 1) < 1e-14


def test_p11_eigensolver_against_high_precision():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11)
    M = crandn(rng, 3, 3)
    M = M + M.conj().T
    lam, U, V = oracle.top_eigvecs(M, 2)
    E, Q = mpmath.eighe(mpmath.matrix(M.tolist()))
    ref = sorted([float(mpmath.re(E[i])) for i in range(3)], reverse=True)
    np.testing.assert_allclose(lam, ref, rtol=1e-13, atol=1e-13)
    for i in range(3):
        np.testing.assert_allclose(M @ V[:, i], lam[i] * V[:, i], atol=1e-13)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(3), atol=1e-14)


# ---------------------------------------------------------------- P12
def test_p12_invariances():
    """Scaling the training data, permuting the stencil or a global phase on
    the test snapshot leave T unchanged (up to rounding)."""
    sc = scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=24, W=24, n_targets=2), seed=12)
    cfg = oracle.OracleConfig(p=3, q=8, n=64)
    st = cfg.training_stencil()
    pix = np.array([[12, 12], [11, 13], [14, 10]])
    base = oracle.kron_stap_pixels(sc.x, pix, cfg)["T"]
    perm = np.random.default_rng(0).permutation(st.shape[0])
    cfg_p = oracle.OracleConfig(p=3, q=8, n=64, stencil=st[perm])
    np.testing.assert_allclose(oracle.kron_stap_pixels(sc.x, pix, cfg_p)["T"], base, rtol=1e-10)
    # scale the training data by 3 and rotate the test snapshot's phase; the
    # pixel is not in its own stencil, so S scales by 9 and U_A, U_B, T stay.
    for i, (r, c) in enumerate(pix):
        x4 = sc.x.astype(np.complex128) * 3.0
        x4[:, r, c, :] = sc.x[:, r, c, :] * np.exp(0.7j)
        t = oracle.kron_stap_pixels(x4, pix[i:i + 1], cfg)["T"][0]
        assert t == pytest.approx(base[i], rel=1e-10)


# ---------------------------------------------------------------- P13
@pytest.mark.parametrize("n,W", [(64, 10), (128, 12), (200, 16), (256, 18)])
def test_p13_default_stencil(n, W):
    st = oracle.default_stencil(n)
    assert st.shape == (n, 2)
    assert oracle.stencil_window(n) == W
    assert len({tuple(t) for t in st}) == n
    assert not any(abs(dr) <= 1 and abs(dc) <= 1 for dr, dc in st)
    assert st.min() >= -W // 2 and st.max() <= W // 2 - 1
    d2 = st[:, 0] ** 2 + st[:, 1] ** 2
    assert np.all(np.diff(d2) >= 0)


def test_p13_valid_region():
    """A pixel is processed iff its whole stencil lies inside the frame (brute force)."""
    for n, H, W in ((64, 64, 64), (200, 40, 33), (256, 18, 30)):
        st = oracle.default_stencil(n)
        r0, r1, c0, c1 = oracle.valid_region(H, W, st)
        rows = [r for r in range(H) if all(0 <= r + dr < H for dr in st[:, 0])]
        cols = [c for c in range(W) if all(0 <= c + dc < W for dc in st[:, 1])]
        assert list(range(r0, r1)) == rows and list(range(c0, c1)) == cols


# ---------------------------------------------------------------- P15
def test_p15_eta_is_monotone():
    """eta_k is non-increasing along Alg. 2 (FP64)."""
    rng = np.random.default_rng(15)
    p, q = 3, 8
    worst = 0.0
    for _ in range(40):
        X = crandn(rng, p * q, 30)
        S = X @ X.conj().T / 30 + 20 * np.kron(rand_psd(rng, p, 1), rand_psd(rng, q, 3))
        R = oracle.rearrange(S, p, q)
        prev = np.inf
        for k in range(1, 8):
            e = oracle.lr_kron(R, p, q, 1, 3, eps=0.0, max_iter=k)["eta"]
            if np.isfinite(prev):
                worst = max(worst, (e - prev) / prev)
            prev = e
    assert worst <= 1e-12


# ---------------------------------------------------------------- edge cases
def test_zero_and_nonfinite_training():
    """Reading R11: zero training gives T = 0; a NaN gives T = NaN, D = 0."""
    cfg = oracle.OracleConfig(p=3, q=8, n=64)
    x = np.zeros((3, 20, 20, 8), np.complex64)
    out = oracle.kron_stap_pixels(x, np.array([[10, 10]]), cfg)
    assert out["T"][0] == 0.0 and out["D"][0] == 0
    x = scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=20, W=20, n_targets=0), 3).x
    x[1, 8, 8, 3] = np.nan
    out = oracle.kron_stap_pixels(x, np.array([[10, 10], [8, 8], [14, 14]]), cfg)
    assert np.isnan(out["T"][0]) and np.isnan(out["T"][1]) and out["D"][0] == 0
    assert np.isfinite(out["T"][2])
    # outside the valid region
    out = oracle.kron_stap_pixels(x, np.array([[2, 2]]), cfg)
    assert out["T"][0] == 0.0 and not out["valid"][0]


def test_rank_b_zero_keeps_temporal_space():
    """r_b = 0 (Sec. 5: U_B = 0 when r_b approaches q) gives F_B = I."""
    rng = np.random.default_rng(16)
    p, q = 3, 5
    UA = np.linalg.qr(crandn(rng, p, 1))[0]
    X = crandn(rng, p, q)
    bs = np.ones(q)
    T = oracle.kron_stap_statistic(X, UA, np.zeros((q, 0)), bs)
    z = (np.eye(p) - proj(UA)) @ X @ bs
    assert T == pytest.approx(np.vdot(z, z).real / q, rel=1e-13)


# ---------------------------------------------------------------- P14
def test_p14_detection_sanity_on_tiny_scene():
    """Integrated target SNR >= pq: most targets inside the valid region are
    detected; false alarms stay near pfa."""
    sc = scenegen.make_scene(scenegen.TINY)
    cfg = oracle.OracleConfig(p=3, q=8, n=64, r_a=1, r_b=3)
    out = oracle.kron_stap_frame(sc.x, cfg)
    r0, r1, c0, c1 = oracle.valid_region(64, 64, cfg.training_stencil())
    inside = [(r, c) for r, c in sc.targets if r0 <= r < r1 and c0 <= c < c1]
    hits = sum(int(out["D_img"][r, c]) for r, c in inside)
    assert hits >= len(inside) - 1
    fa = int(out["D_img"].sum()) - hits
    assert fa <= 3
    assert np.all(out["iters"][out["valid"]] <= 4)


# ---------------------------------------------------------------- SCM (Eq. (2))
def test_scm_hermitian_psd_trace_and_constant_field():
    """S is Hermitian PSD with trace = mean snapshot energy; a frame whose
    training snapshots all equal v gives S = v v^H (top eigenpair v, ||v||^2)."""
    sc = scenegen.make_scene(scenegen.SceneSpec(p=3, q=8, H=24, W=24, n_targets=0), seed=21)
    st = oracle.default_stencil(64)
    rows, cols = np.array([12, 13]), np.array([11, 12])
    S = oracle.sample_covariance(sc.x, rows, cols, st)
    for k in range(2):
        np.testing.assert_allclose(S[k], S[k].conj().T, atol=1e-12 * np.abs(S[k]).max())
        assert np.linalg.eigvalsh(S[k]).min() >= -1e-10 * np.abs(S[k]).max()
        energy = np.mean([np.sum(np.abs(sc.x[:, rows[k] + dr, cols[k] + dc, :].astype(complex)) ** 2)
                          for dr, dc in st])
        assert np.trace(S[k]).real == pytest.approx(energy, rel=1e-12)
    rng = np.random.default_rng(22)
    V = crandn(rng, 3, 8)
    x = np.broadcast_to(V[:, None, None, :], (3, 24, 24, 8)).astype(np.complex128)
    S = oracle.sample_covariance(x, np.array([12]), np.array([12]), st)[0]
    lam, U = np.linalg.eigh(S)
    v = V.reshape(24)                              # vec(V^T): channel-major
    assert lam[-1] == pytest.approx(np.vdot(v, v).real, rel=1e-12)
    assert abs(abs(np.vdot(U[:, -1], v)) / np.linalg.norm(v) - 1) < 1e-12
    assert np.all(np.abs(lam[:-1]) <= 1e-12 * lam[-1])


# ---------------------------------------------------------------- R9 (graded set)
def test_relative_gap_on_known_spectra():
    """The truncation gap that decides which pixels are graded: for a known
    spectrum (4, 3, 1, 0.5) the gaps after ranks 1, 2, 3 are 1/4, 2/4 and
    0.5/4 of the largest eigenvalue (hand-computed constants), both on the
    sorted eigenvalues directly and after a random unitary rotation of the
    diagonal matrix through the oracle's eigensolver; ranks 0 and 4 (no
    truncation) count as a full gap."""
    lam = np.array([4.0, 3.0, 1.0, 0.5])
    expect = {1: 0.25, 2: 0.5, 3: 0.125}
    for r, g in expect.items():
        assert oracle.relative_gaps(lam, r) == pytest.approx(g, rel=1e-15)
    rng = np.random.default_rng(31)
    Q = np.linalg.qr(crandn(rng, 4, 4))[0]
    M = (Q * lam) @ Q.conj().T
    ev, _, _ = oracle.top_eigvecs(M, 2)
    for r, g in expect.items():
        assert oracle.relative_gaps(ev, r) == pytest.approx(g, rel=1e-12)
    assert oracle.relative_gaps(lam, 0) == 1.0
    assert oracle.relative_gaps(lam, 4) == 1.0
    # batched rows keep their own gaps
    batch = np.array([[4.0, 3.0, 1.0, 0.5], [2.0, 2.0, 2.0, 0.0], [1.0, 0.0, 0.0, 0.0]])
    np.testing.assert_allclose(oracle.relative_gaps(batch, 2), [0.5, 0.0, 0.0], rtol=1e-15, atol=0)
    np.testing.assert_allclose(oracle.relative_gaps(batch, 3), [0.125, 1.0, 0.0], rtol=1e-15, atol=0)
    np.testing.assert_array_equal(oracle.relative_gaps(batch, 0), np.ones(3))


def test_relative_gap_flags_a_tie_at_the_truncation():
    """A pixel whose space factor has two equal leading eigenvalues cannot be
    graded at rank 1 (several subspaces are correct), while a clear gap passes
    the 1e-3 bar."""
    rng = np.random.default_rng(32)
    Q = np.linalg.qr(crandn(rng, 3, 3))[0]
    tie, _, _ = oracle.top_eigvecs((Q * np.array([2.0, 2.0, 0.1])) @ Q.conj().T, 1)
    clear, _, _ = oracle.top_eigvecs((Q * np.array([2.0, 1.0, 0.1])) @ Q.conj().T, 1)
    assert oracle.relative_gaps(tie, 1) < 1e-12
    assert oracle.relative_gaps(clear, 1) == pytest.approx(0.5, rel=1e-12)
