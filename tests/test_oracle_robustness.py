"""Pins of the robustness oracle (`oracle/robustness.py`): the LR-STAP
baseline, the true SIRV covariance and the SINR of Eqs. (21)-(23), each fixed
by something other than the oracle itself: closed forms (identity filter,
Sherman-Morrison for a rank-one clutter, the Kronecker eigen-relation), the
Cauchy-Schwarz bound that makes Sigma^-1 optimal, an exactly Kronecker
training set whose top eigenvectors are known, and brute-force power
iteration on tiny inputs.  The SIRV generator's second moments are checked
against the model covariance by Monte Carlo."""
import numpy as np
import pytest

import oracle
import oracle.robustness as RB
import scenegen


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def _orth(rng, n, r):
    q, _ = np.linalg.qr(_cn(rng, (n, r)))
    return q[:, :r]


# ------------------------------------------------------------ true covariance
def test_true_covariance_kronecker_eigen_relation():
    """(A (x) B)(u (x) v) = (A u) (x) (B v): every u_i (x) v_j is an
    eigenvector with eigenvalue tau2 lamA_i lamB_j + sigma2, and vectors
    orthogonal to all of them see sigma2 alone."""
    rng = _rng(1)
    p, q = 3, 5
    UA, UB = _orth(rng, p, 2), _orth(rng, q, 3)
    la, lb = np.array([3.0, 0.7]), np.array([10.0, 4.0, 0.5])
    S = RB.true_covariance(UA, la, UB, lb, sigma2=0.8, tau2_mean=1.7)
    for i in range(2):
        for j in range(3):
            v = np.kron(UA[:, i], UB[:, j])
            assert np.allclose(S @ v, (1.7 * la[i] * lb[j] + 0.8) * v, atol=1e-12)
    C = np.kron(UA, UB)
    z = _cn(rng, p * q)
    z -= C @ (C.conj().T @ z)
    assert np.allclose(S @ z, 0.8 * z, atol=1e-12)
    assert np.allclose(S, S.conj().T)


def test_sirv_generator_second_moments():
    """Pixels of a texture scene (no targets) have covariance
    E[tau^2] A (x) B + I in the vec(X^T) order, and the texture has
    E[tau^2] = 1, Var[tau^2] = 1/nu (Gamma(nu, 1/nu))."""
    spec = scenegen.SirvSpec(p=2, q=3, H=200, W=200, r_a=1, r_b=2, cnr_db=10.0, texture_nu=0.8, n_test=0)
    sc = scenegen.make_sirv_scene(spec, seed=77)
    v = sc.x.transpose(1, 2, 0, 3).reshape(-1, 6).astype(np.complex128)
    S_hat = v.T @ v.conj() / v.shape[0]
    S = RB.true_covariance(sc.UA, sc.lamA, sc.UB, sc.lamB, sc.sigma2, sc.tau2_mean)
    assert np.linalg.norm(S_hat - S) / np.linalg.norm(S) < 0.05
    t = sc.tau2.ravel()
    assert abs(t.mean() - 1.0) < 0.03
    assert abs(t.var() - 1.0 / 0.8) < 0.15
    # texture is per pixel: clutter power of a pixel scales with its tau^2
    hi, lo = t > np.quantile(t, 0.9), t < np.quantile(t, 0.1)
    pw = np.sum(np.abs(v) ** 2, axis=1)
    assert pw[hi].mean() > 5 * pw[lo].mean()


def test_sirv_corruption_inside_training_window():
    spec = scenegen.SirvSpec(p=3, q=8, H=64, W=64, texture_nu=None, n_test=6, n_corrupt=4, radius=6, inner=2)
    sc = scenegen.make_sirv_scene(spec, seed=3)
    assert sc.corrupt.shape == (24, 2)
    for t in range(6):
        c = sc.corrupt[4 * t:4 * t + 4]
        d = np.abs(c - sc.test_pixels[t][None]).max(axis=1)
        assert np.all((d >= 2) & (d <= 6))
        assert len({tuple(e) for e in c}) == 4


# ------------------------------------------------------------------ SINR
def test_sinr_identity_filter_white_noise():
    rng = _rng(2)
    d = _cn(rng, 12)
    S = 0.5 * np.eye(12)
    assert np.isclose(RB.sinr_out(d, d, S), np.vdot(d, d).real / 0.5)
    assert np.isclose(RB.sinr_optimal(d, S), np.vdot(d, d).real / 0.5)
    F = np.eye(12)[None]
    a, b = np.exp(1j * 0.3 * np.arange(3)), np.exp(2j * np.pi * 0.1 * np.arange(4))
    assert np.allclose(RB.sinr_loss_grid(F, [a], [b], S), 1.0)


def test_sinr_optimal_rank_one_sherman_morrison():
    rng = _rng(3)
    n = 10
    u = _orth(rng, n, 1)[:, 0]
    lam, s2 = 50.0, 2.0
    S = lam * np.outer(u, u.conj()) + s2 * np.eye(n)
    d = _cn(rng, n)
    closed = (np.vdot(d, d).real - lam / (lam + s2) * abs(np.vdot(u, d)) ** 2) / s2
    assert np.isclose(RB.sinr_optimal(d, S), closed, rtol=1e-12)
    # identity filter: |d|^4 / (d^H S d)
    dd = np.vdot(d, d).real
    assert np.isclose(RB.sinr_out(d, d, S), dd ** 2 / (lam * abs(np.vdot(u, d)) ** 2 + s2 * dd), rtol=1e-12)


def test_sinr_loss_bounds_and_optimum():
    """Loss of Sigma^-1 is 1; of any filter, at most 1 (Cauchy-Schwarz)."""
    rng = _rng(4)
    p, q = 3, 4
    S = RB.true_covariance(_orth(rng, p, 1), [2.0], _orth(rng, q, 2), [300.0, 80.0])
    a_grid = [np.exp(1j * t * np.arange(p)) for t in (0.0, 0.7, 2.0)]
    b_grid = [np.exp(2j * np.pi * f * np.arange(q)) for f in (-0.3, 0.0, 0.2)]
    Fopt = np.linalg.inv(S)[None]
    assert np.allclose(RB.sinr_loss_grid(Fopt, a_grid, b_grid, S), 1.0, atol=1e-12)
    G = _cn(rng, (20, p * q, p * q))
    L = RB.sinr_loss_grid(G, a_grid, b_grid, S)
    assert np.all(L <= 1.0 + 1e-12) and np.all(L >= 0.0) and L.max() < 1.0


def test_sinr_loss_exact_subspaces():
    """With the true subspaces, Kron-STAP passes a target outside both
    clutter subspaces untouched and removes all clutter from it: loss 1.
    A target inside the clutter subspace is cancelled (F d = 0)."""
    rng = _rng(5)
    p, q = 3, 6
    UA, UB = _orth(rng, p, 1), _orth(rng, q, 2)
    S = RB.true_covariance(UA, [3.0], UB, [500.0, 120.0])
    a = _cn(rng, p)
    a -= UA @ (UA.conj().T @ a)
    b = _cn(rng, q)
    b -= UB @ (UB.conj().T @ b)
    for kind in ("kron", "classical"):
        F = RB.filters(kind, U_A=UA[None], U_B=UB[None])
        assert np.isclose(RB.sinr_loss_grid(F, [a], [b], S)[0, 0, 0], 1.0, rtol=1e-10)
    U = np.kron(UA, UB)[None]
    assert np.isclose(RB.sinr_loss_grid(RB.filters("lrstap", U=U), [a], [b], S)[0, 0, 0], 1.0, rtol=1e-10)
    Fk = RB.filters("kron", U_A=UA[None], U_B=UB[None])
    assert np.linalg.norm(Fk[0] @ RB.steering(UA[:, 0], UB[:, 1])) < 1e-12


# ---------------------------------------------------------------- LR-STAP
def _frame(rng, p, q, H, W):
    return _cn(rng, (p, H, W, q)).astype(np.complex64)


def test_lrstap_rank_zero_is_matched_filter():
    """r = 0: F = I, T = ||E^H x||^2 / ||b||^2 = sum_i |X[i] . conj(b)|^2 / ||b||^2."""
    rng = _rng(6)
    p, q = 3, 4
    x = _frame(rng, p, q, 24, 24)
    b = np.exp(2j * np.pi * 0.15 * np.arange(q))
    cfg = oracle.OracleConfig(p=p, q=q, n=40, b_steer=b)
    pix = np.array([[12, 12], [13, 11], [11, 14]])
    out = RB.lr_stap_pixels(x, pix, cfg, r=0)
    X = x[:, pix[:, 0], pix[:, 1], :].transpose(1, 0, 2).astype(np.complex128)
    ref = np.sum(np.abs(X @ np.conj(b)) ** 2, axis=1) / np.vdot(b, b).real
    assert np.allclose(out["T"], ref, rtol=1e-12)


def test_lrstap_full_rank_cancels_everything():
    rng = _rng(7)
    x = _frame(rng, 2, 3, 24, 24)
    cfg = oracle.OracleConfig(p=2, q=3, n=40)
    out = RB.lr_stap_pixels(x, np.array([[12, 12]]), cfg, r=6)
    assert abs(out["T"][0]) < 1e-9


def test_lrstap_exact_kronecker_training_equals_classical_projector():
    """Training vectors u_a (x) v_m give S = (u_a u_a^H) (x) B_n exactly, so
    the top r_b eigenvectors of S are u_a (x) (top eigenvectors of B_n) and
    LR-STAP's filter is the joint projector of Eq. (24) built from u_a and
    B_n's eigenvectors: the statistics agree."""
    rng = _rng(8)
    p, q, rb = 3, 5, 2
    H = W = 30
    x = _frame(rng, p, q, H, W) * 0.1
    ua = _orth(rng, p, 1)[:, 0]
    cfg = oracle.OracleConfig(p=p, q=q, n=60, r_a=1, r_b=rb)
    st = cfg.training_stencil()
    r0, c0 = 15, 15
    # a clutter-like B: strong rank-2 part plus a weak floor, drawn through v_m
    Vb = _orth(rng, q, q)
    scales = np.array([30.0, 12.0, 1.0, 0.6, 0.3])
    vs = []
    for (dr, dc) in st:
        v = Vb @ (np.sqrt(scales) * _cn(rng, q))
        vs.append(v)
        x[:, r0 + dr, c0 + dc, :] = np.outer(ua, v).astype(np.complex64)
    vs = np.array(vs, dtype=np.complex64).astype(np.complex128)
    Bn = (vs.T @ vs.conj()) / len(st)
    lb, Ub = np.linalg.eigh(Bn)
    UB = Ub[:, ::-1][:, :rb]
    out = RB.lr_stap_pixels(x, np.array([[r0, c0]]), cfg, r=rb)
    from oracle.variants import filter_matrix, glrt_explicit
    F = filter_matrix(ua.reshape(1, p, 1), UB.reshape(1, q, rb), "classical")
    Xt = x[:, [r0], [c0], :].transpose(1, 0, 2).astype(np.complex128)
    T_ref, _ = glrt_explicit(F, Xt, np.ones(q))
    P = out["U"][0] @ out["U"][0].conj().T
    P_ref = np.kron(np.outer(ua, ua.conj()), UB @ UB.conj().T)
    assert np.linalg.norm(P - P_ref) < 1e-5
    assert np.isclose(out["T"][0], T_ref[0], rtol=1e-5)


def test_lrstap_brute_force_power_iteration():
    """Tiny case: the projector onto the top-r eigenvectors of the sample
    covariance, found by power iteration with deflation on S formed by an
    explicit loop over the training vectors."""
    rng = _rng(9)
    p, q, r = 2, 3, 2
    x = _frame(rng, p, q, 20, 20)
    x[:, :, :, 0] *= 6.0
    x[1, :, :, 2] *= 3.0
    cfg = oracle.OracleConfig(p=p, q=q, n=30)
    rc = (10, 9)
    S = np.zeros((6, 6), complex)
    for dr, dc in cfg.training_stencil():
        X = x[:, rc[0] + dr, rc[1] + dc, :].astype(np.complex128)
        v = np.array([X[i, k] for i in range(p) for k in range(q)])   # vec(X^T)
        S += np.outer(v, v.conj())
    S /= cfg.n
    U = []
    M = S.copy()
    for _ in range(r):
        v = np.ones(6, complex)
        for _ in range(5000):
            v = M @ v
            v /= np.linalg.norm(v)
        lam = np.vdot(v, M @ v).real
        U.append(v)
        M = M - lam * np.outer(v, v.conj())
    U = np.array(U).T
    out = RB.lr_stap_pixels(x, np.array([rc]), cfg, r=r)
    assert np.linalg.norm(out["U"][0] @ out["U"][0].conj().T - U @ U.conj().T) < 1e-8
    lam_all = np.sort(np.linalg.eigvalsh(S))[::-1]
    assert np.allclose(out["lam"][0], lam_all[:r + 1], rtol=1e-10)


def test_lrstap_invalid_pixels_zero():
    rng = _rng(10)
    x = _frame(rng, 2, 3, 20, 20)
    cfg = oracle.OracleConfig(p=2, q=3, n=30)
    out = RB.lr_stap_pixels(x, np.array([[0, 0], [10, 10]]), cfg)
    assert not out["valid"][0] and out["valid"][1]
    assert out["T"][0] == 0 and np.all(out["U"][0] == 0)


# ---------------------------------------------------------------- mutants
MUTANTS = {
    "smallest eigenvalues": ("lr_stap_pixels", "lam, V = lam[:, ::-1], V[:, :, ::-1]", "lam, V = lam, V"),
    "projector kept instead of removed": (
        "lrstap_filter", "return np.eye(pq)[None] - np.matmul(U, np.conj(np.swapaxes(U, -1, -2)))",
        "return np.matmul(U, np.conj(np.swapaxes(U, -1, -2)))"),
    "noise term dropped": ("true_covariance", "+ sigma2 * np.eye(A.shape[0] * B.shape[0])", "+ 0.0"),
    "texture power ignored": ("true_covariance", "return tau2_mean * np.kron(A, B)", "return np.kron(A, B)"),
    "steering order swapped": ("steering", "np.kron(np.asarray(a, np.complex128), np.asarray(b, np.complex128))",
                               "np.kron(np.asarray(b, np.complex128), np.asarray(a, np.complex128))"),
    "SINR without conjugate": ("sinr_out", 'num = np.abs(np.einsum("...i,i->...", np.conj(w), d)) ** 2',
                               'num = np.abs(np.einsum("...i,i->...", w, d)) ** 2'),
    "optimum without inverse": ("sinr_optimal", "np.linalg.solve(Sigma, d)", "Sigma @ d"),
}


def _pins():
    return [test_true_covariance_kronecker_eigen_relation, test_sirv_generator_second_moments,
            test_sinr_identity_filter_white_noise, test_sinr_optimal_rank_one_sherman_morrison,
            test_sinr_loss_bounds_and_optimum, test_sinr_loss_exact_subspaces, test_lrstap_rank_zero_is_matched_filter,
            test_lrstap_full_rank_cancels_everything, test_lrstap_exact_kronecker_training_equals_classical_projector,
            test_lrstap_brute_force_power_iteration]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_robustness_mutant_fails_a_pin(name, monkeypatch):
    import inspect
    import textwrap
    fn_name, old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(getattr(RB, fn_name)))
    assert old in src, name
    ns = dict(RB.__dict__)
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), ns)
    monkeypatch.setattr(RB, fn_name, ns[fn_name])
    # functions that call the mutated one through the module see the mutant
    for other in ("lr_stap_pixels", "true_covariance", "steering", "sinr_out", "sinr_optimal", "lrstap_filter",
                  "filters", "sinr_loss_grid"):
        if other != fn_name:
            src2 = textwrap.dedent(inspect.getsource(getattr(RB, other)))
            ns2 = dict(RB.__dict__)
            ns2[fn_name] = ns[fn_name]
            exec(compile(src2, f"<rebound {other}>", "exec"), ns2)
            monkeypatch.setattr(RB, other, ns2[other])
    failed = 0
    with np.errstate(all="ignore"):
        for pin in _pins():
            try:
                pin()
            except (AssertionError, np.linalg.LinAlgError, ValueError):
                failed += 1
    assert failed >= 1, f"mutant '{name}' passes every pin"
