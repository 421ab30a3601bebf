"""FP64 oracle of the robustness evaluation (test infrastructure only, like
the rest of this package): the unstructured low-rank STAP baseline and the
output SINR of a filter against the true clutter-plus-noise covariance.

What it computes:

  * LR-STAP (the classical low-rank STAP the Kronecker methods are compared
    with, Sec. 1): per pixel, the sample covariance S of Eq. (2) over the same
    training stencil as the Kron-STAP oracle, the eigenvectors U of its r
    largest eigenvalues (a full Hermitian eigendecomposition), the filter
    F = I - U U^H, and the statistic of reading V1 (`variants.py`) for that
    filter;
  * the true covariance of the SIRV model: Sigma = E[tau^2] A (x) B + sigma^2 I
    (Eqs. (5) and (7), with the speckle covariance A (x) B of Eq. (9));
  * the output SINR of Eq. (21) for a filter w = F d (Eq. (23)) and target
    steering d, with |alpha| = 1, and the SINR loss against the optimal filter
    F = Sigma^-1 of Eq. (22): loss = SINR_out(F d) / SINR_out(Sigma^-1 d).

Readings:

  S1  LR-STAP rank: r = r_a r_b by default, the rank of the Kronecker clutter
      model A (x) B the scenes are drawn from; any 0 <= r <= pq is accepted.
      The eigenvalues are taken in decreasing algebraic order; with r = 0 the
      filter is the identity.  Its detection threshold, like the classical
      filter's (V4), is the Gamma(p, 1) quantile.
  S2  SINR with |alpha| = 1: SINR_out(w) = |w^H d|^2 / (w^H Sigma w); the
      optimum d^H Sigma^-1 d is reached by w = Sigma^-1 d (Cauchy-Schwarz), so
      the loss lies in [0, 1].  A filter with w = 0 has loss 0.
  S3  Steering d = a(theta) (x) b(f) with a_i = exp(j i theta) (Eq. (8)) and
      b_k = exp(2 pi j f k), a constant Doppler shift f in cycles per sample.

Everything is evaluated from explicit pq x pq matrices (dense Sigma, its
inverse by a linear solve, dense filters), never from the factored forms the
GPU kernels use.
"""
from __future__ import annotations

import numpy as np

from .kron_stap import OracleConfig, sample_covariance, snapshots, valid_region
from .variants import filter_matrix, glrt_explicit


def lr_stap_pixels(x: np.ndarray, pixels: np.ndarray, cfg: OracleConfig, r: int = -1) -> dict:
    """LR-STAP on pixels [(r, c), ...] of frame x [p][H][W][q] (reading S1).
    Returns T [N], U [N, pq, r], lam [N, min(r + 1, pq)] (the r + 1 largest
    eigenvalues of S, decreasing), valid [N] (whole stencil inside; T = 0 and
    U = 0 elsewhere)."""
    p, H, W, q = x.shape
    pq = p * q
    if r < 0:
        r = cfg.r_a * cfg.r_b
    if not 0 <= r <= pq:
        raise ValueError("LR-STAP rank outside [0, pq]")
    pix = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    N = pix.shape[0]
    st = cfg.training_stencil()
    r0, r1, c0, c1 = valid_region(H, W, st)
    valid = (pix[:, 0] >= r0) & (pix[:, 0] < r1) & (pix[:, 1] >= c0) & (pix[:, 1] < c1)
    nl = min(r + 1, pq)
    out = dict(T=np.zeros(N), U=np.zeros((N, pq, r), np.complex128), lam=np.zeros((N, nl)), valid=valid)
    ids = np.nonzero(valid)[0]
    if ids.size == 0:
        return out
    rows, cols = pix[ids, 0], pix[ids, 1]
    S = sample_covariance(x, rows, cols, st)                 # Eq. (2)
    lam, V = np.linalg.eigh(S)                               # increasing
    lam, V = lam[:, ::-1], V[:, :, ::-1]                     # decreasing
    U = V[:, :, :r]
    F = np.eye(pq)[None] - np.matmul(U, np.conj(np.swapaxes(U, -1, -2)))
    T, _ = glrt_explicit(F, snapshots(x, rows, cols), cfg.temporal_steering())
    out["T"][ids] = T
    out["U"][ids] = U
    out["lam"][ids] = lam[:, :nl]
    return out


def true_covariance(UA: np.ndarray, lamA: np.ndarray, UB: np.ndarray, lamB: np.ndarray,
                    sigma2: float = 1.0, tau2_mean: float = 1.0) -> np.ndarray:
    """Sigma = E[tau^2] A (x) B + sigma^2 I with A = UA diag(lamA) UA^H and
    B = UB diag(lamB) UB^H (Eqs. (5), (7), (9)); dense pq x pq."""
    A = (np.asarray(UA) * np.asarray(lamA)) @ np.conj(np.asarray(UA)).T
    B = (np.asarray(UB) * np.asarray(lamB)) @ np.conj(np.asarray(UB)).T
    return tau2_mean * np.kron(A, B) + sigma2 * np.eye(A.shape[0] * B.shape[0])


def steering(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """d = a (x) b (reading S3), in the vec(X^T) order."""
    return np.kron(np.asarray(a, np.complex128), np.asarray(b, np.complex128))


def sinr_out(w: np.ndarray, d: np.ndarray, Sigma: np.ndarray) -> np.ndarray:
    """Eq. (21) with |alpha| = 1, for filters w [..., pq] and steering d [pq]."""
    num = np.abs(np.einsum("...i,i->...", np.conj(w), d)) ** 2
    den = np.real(np.einsum("...i,ij,...j->...", np.conj(w), Sigma, w))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def sinr_optimal(d: np.ndarray, Sigma: np.ndarray) -> float:
    """SINR of the optimal filter Sigma^-1 d (Eq. (22)): d^H Sigma^-1 d."""
    return float(np.real(np.vdot(d, np.linalg.solve(Sigma, d))))


def lrstap_filter(U: np.ndarray) -> np.ndarray:
    """F = I - U U^H for bases U [N, pq, r]."""
    pq = U.shape[1]
    return np.eye(pq)[None] - np.matmul(U, np.conj(np.swapaxes(U, -1, -2)))


def filters(kind: str, U_A=None, U_B=None, U=None) -> np.ndarray:
    """Dense filters [N, pq, pq]: 'kron' (Eq. (25)), 'classical' (Eq. (24))
    from U_A [N, p, r_a] and U_B [N, q, r_b]; 'lrstap' from U [N, pq, r]."""
    if kind == "lrstap":
        return lrstap_filter(np.asarray(U, np.complex128))
    return filter_matrix(np.asarray(U_A, np.complex128), np.asarray(U_B, np.complex128), kind)


def sinr_loss_grid(F: np.ndarray, a_grid: np.ndarray, b_grid: np.ndarray, Sigma: np.ndarray) -> np.ndarray:
    """SINR loss (reading S2) of filters F [N, pq, pq] for every steering
    d = a (x) b, a in a_grid [na, p], b in b_grid [nb, q].  [N, na, nb]"""
    N = F.shape[0]
    na, nb = len(a_grid), len(b_grid)
    out = np.zeros((N, na, nb))
    for i in range(na):
        for j in range(nb):
            d = steering(a_grid[i], b_grid[j])
            w = np.matmul(F, d)                               # Eq. (23): w = F d
            out[:, i, j] = sinr_out(w, d, Sigma) / sinr_optimal(d, Sigma)
    return out
