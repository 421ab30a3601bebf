"""Pins of the large-covariance oracle (`oracle/large_q.py`, Sec. 6.1): the
rearrangement of a snapshot covariance is a sum of Kronecker products of the
snapshots with their conjugates (Algorithm 1 checked at large q), exact
recovery from an exactly Kronecker snapshot set, the full-rank case against
the leading singular pair of R (a LAPACK SVD of the small Gram form), and the
structure of the timing workload's generator."""
import numpy as np
import pytest

import oracle
import oracle.large_q as LQ
import scenegen


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


@pytest.mark.parametrize("p,q,n", [(3, 40, 5), (2, 300, 3), (6, 25, 4)])
def test_rearranged_snapshot_covariance_is_a_sum_of_kronecker_products(p, q, n):
    """Algorithm 1 on S = (1/n) sum x_m x_m^H gives (1/n) sum conj(X_m) (x) X_m."""
    rng = np.random.default_rng(p * 1000 + q + n)
    X = crandn(rng, n, p, q)
    R = oracle.rearrange(LQ.snapshot_covariance(X), p, q)
    K = sum(np.kron(np.conj(X[m]), X[m]) for m in range(n)) / n
    np.testing.assert_allclose(R, K, atol=1e-14)


def test_snapshot_covariance_is_eq2():
    rng = np.random.default_rng(3)
    X = crandn(rng, 4, 3, 7)
    S = LQ.snapshot_covariance(X)
    ref = sum(np.outer(X[m].reshape(-1), np.conj(X[m].reshape(-1))) for m in range(4)) / 4
    np.testing.assert_allclose(S, ref, atol=1e-15)
    np.testing.assert_allclose(S, S.conj().T, atol=1e-15)


def test_exact_kronecker_snapshots_are_recovered_in_one_iteration():
    """X_m = u w_m^T: S = (u u^H) (x) (1/n sum w_m w_m^H) exactly, so eta = 0
    and A-hat (x) B-hat = S after one iteration."""
    rng = np.random.default_rng(4)
    p, q, n = 3, 120, 5
    u = crandn(rng, p)
    X = np.stack([np.outer(u, crandn(rng, q)) for _ in range(n)])
    out = LQ.lr_kron_snapshots(X, r_a=1, eps=0.0, max_iter=1)
    assert out["eta"] < 1e-12 and out["iters"] == 1
    S = LQ.snapshot_covariance(X)
    np.testing.assert_allclose(np.kron(out["A"], out["B"]), S, atol=1e-10 * np.abs(S).max())


def test_full_rank_fit_is_the_leading_singular_pair():
    """r_a = p: Algorithm 2 is power iteration on R, converging to the
    nearest Kronecker product, the leading singular pair of R (SVD)."""
    rng = np.random.default_rng(6)
    p, q, n = 3, 60, 5
    X = crandn(rng, n, p, q)
    out = LQ.lr_kron_snapshots(X, r_a=p, eps=0.0, max_iter=400)
    R = oracle.rearrange(LQ.snapshot_covariance(X), p, q)
    U, s, Vh = np.linalg.svd(R, full_matrices=False)
    best = s[0] * np.outer(U[:, 0], Vh[0])
    from oracle.kron_stap import _vec
    fit = np.outer(_vec(out["A"]), _vec(out["B"]))
    np.testing.assert_allclose(fit, best, atol=1e-8 * s[0])


def test_timing_workload_generator():
    """Rank-one A (x) I_q + I: the population covariance of the snapshots, in
    the mean over many draws, has the Kronecker structure of Sec. 6.1."""
    X = scenegen.large_q_snapshots(3, 6, 4000, seed=7)
    S = LQ.snapshot_covariance(X)
    R = oracle.rearrange(S, 3, 6)
    s = np.linalg.svd(R, compute_uv=False)
    assert s[1] < 0.05 * s[0]   # nearly one Kronecker term
    lam = np.linalg.eigvalsh(S)[::-1]
    assert lam[5] > 10 * lam[6]  # q = 6 strong directions (rank-one A times I_6) over the noise
