"""FP64 oracle of LR-Kron on one large covariance (test infrastructure only).

The paper times Algorithm 2 alone on single covariances with many azimuth
samples: p = 3 or 6 channels, q up to 2500, n = 5 training snapshots, a
rank-one space factor and an identity time factor (Sec. 6.1, Fig. time3),
at tolerances 1e-4 and 1e-6.  This module runs that estimation literally:
the pq x pq sample covariance of the snapshots (Sec. 1.1, Eq. (2)), its
rearrangement by Algorithm 1, and Algorithm 2 with the stop rule of reading R6,
returning A-hat, the final time factor B-hat (the half-step of reading R7,
Hermitian part, untruncated: r_b = q as in the timing experiment), eta and
the iteration count.  Everything goes through `kron_stap.py`; nothing here is
shared with the GPU path.
"""
from __future__ import annotations

import numpy as np

from .kron_stap import lr_kron, rearrange


def snapshot_covariance(X: np.ndarray) -> np.ndarray:
    """S = (1/n) sum_m x_m x_m^H with x_m = vec(X_m^T) (Eq. (2), reading R1);
    X [n, p, q] -> S [pq, pq] complex128."""
    X = np.asarray(X, dtype=np.complex128)
    n, p, q = X.shape
    V = X.reshape(n, p * q)               # row m is vec(X_m^T): V[m, i q + j] = X_m[i, j]
    return (V.T @ V.conj()) / n


def lr_kron_snapshots(X: np.ndarray, r_a: int = 1, eps: float = 1e-6, min_iter: int = 2,
                      max_iter: int = 50) -> dict:
    """Algorithm 2 on R(S) for the snapshots X [n, p, q]: returns A (p x p),
    B (q x q, Hermitian part of the final half-step), eta, iters, and the
    norms ||R||_F, ||a||, ||b||."""
    X = np.asarray(X, dtype=np.complex128)
    n, p, q = X.shape
    S = snapshot_covariance(X)
    R = rearrange(S, p, q)
    est = lr_kron(R, p, q, r_a, q, eps, min_iter, max_iter, truncate_b=False)
    return dict(A=est["A"], B=est["B"], U_A=est["U_A"], eta=float(est["eta"]), iters=int(est["iters"]),
                lam_A=est["lam_A"], normR=float(np.linalg.norm(R)))
