"""FP64 oracle of the filter and statistic variants and of multipass change
detection (test infrastructure only, like the rest of this package).

What it computes, per pixel, on top of the single-pass estimator of
`kron_stap.py` (sample covariance, Algorithm 1, Algorithm 2):

  * the filter F of Sec. 5 as an explicit pq x pq matrix, either the
    Kron-STAP projector (I - U_A U_A^H) (x) (I - U_B U_B^H) of Eq. (25) or the
    classical joint projector I - U_A U_A^H (x) U_B U_B^H of Eq. (24);
  * the statistic of Sec. 6.3 (Eq. (26)) for that filter: the largest
    normalised output |d^H F x|^2 / (d^H F d) over spatial steerings h with
    d = h (x) b, optionally maximised over a bank of temporal steering vectors
    (the Doppler bins d_i of Sec. 6.3), with the index of the best bin;
  * the enhancement image of Sec. 6.3: the Kron-STAP intensity divided by the
    intensity of the original single-antenna SAR image at the same bin;
  * multipass frames (Sec. 3): K registered passes stacked into Kp channels,
    a rank-K space factor, and the non-coherent change detection of Sec. 6.4:
    each pass's image reformed from the filtered data and the magnitudes
    subtracted.

Everything is evaluated from the explicit matrices (the filter, the steering
matrix E = I (x) b), never from the closed forms the GPU kernels use.

Readings (in addition to R1-R11 of `kron_stap.py`):

  V1  For any filter F the statistic is max over h of |d^H F x|^2/(d^H F d)
      with d = h (x) b = E h, E = I_p (x) b.  With u = E^H F x and
      G = E^H F E this is the largest generalised Rayleigh quotient,
      u^H G^+ u, where G^+ inverts the eigenvalues of G above 1e-12 ||b||^2
      and drops the rest (u lies in the range of G for both filters).  Fixed
      spatial steering h: |h^H u|^2 / (h^H G h), 0 where h^H G h is below
      1e-12 ||h||^2 ||b||^2.
  V2  Doppler bank of M bins: b_m[k] = exp(2 pi j ((m k) mod M) / M),
      m = 0..M-1.  The pixel statistic is the maximum over the bank, the bin
      its first maximiser; D = T > tau with tau the single-bin threshold.
  V3  Enhancement: E = T / I_SAR with I_SAR = |sum_k X[0, k] conj(b_k)|^2 /
      ||b||^2, the matched-filter intensity of channel 0 at the same bin
      (unit mean under white noise); E = 0 where I_SAR = 0.
  V4  Classical filter threshold: under white noise with exact subspaces its
      statistic is Gamma(p, 1), so tau defaults to that quantile.
  V5  Multipass: pass k occupies channels k p .. k p + p - 1 of the stacked
      frame; the estimator runs on the Kp-channel frame with r_a = K.  Pass
      k's image is the largest output over unit spatial steerings supported on
      its channels, normalised by the temporal term b^H F_B b as in reading R9:
      T_k = ||u_k||^2 / (b^H F_B b) with u_k the pass-k rows of u (V1).
      The change image of pass k >= 1 against the reference pass 0 is
      C_k = sqrt(T_k) - sqrt(T_0).  Only the Kron-STAP filter is combined with
      several passes.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .kron_stap import (OracleConfig, gamma_upper_quantile, lr_kron, rearrange, sample_covariance, snapshots,
                        valid_region)


@dataclasses.dataclass
class VariantConfig(OracleConfig):
    filter: str = "kron"        # "kron" (Eq. (25)) or "classical" (Eq. (24))
    nbank: int = 0              # 0: the single temporal steering b_steer; M > 0: M Doppler bins (V2)
    passes: int = 1             # K registered passes stacked into p = K * p_pass channels (V5)

    def threshold(self) -> float:
        if self.tau > 0:
            return float(self.tau)
        dof = self.p if self.filter == "classical" else self.p - self.r_a
        return gamma_upper_quantile(dof, self.pfa)

    def steering_set(self) -> np.ndarray:
        """[M, q] temporal steering vectors tried per pixel."""
        if self.nbank > 0:
            return doppler_bank(self.q, self.nbank)
        return self.temporal_steering()[None, :]


def doppler_bank(q: int, M: int) -> np.ndarray:
    """b_m[k] = exp(2 pi j ((m k) mod M) / M) for m < M, k < q (reading V2)."""
    k = np.arange(q)
    m = np.arange(M)
    return np.exp(2j * np.pi * (((m[:, None] * k[None, :]) % M) / M))


def projector(U: np.ndarray) -> np.ndarray:
    """U U^H for orthonormal bases U [N, m, r] (r may be 0)."""
    return np.matmul(U, np.conj(np.swapaxes(U, -1, -2)))


def filter_matrix(U_A: np.ndarray, U_B: np.ndarray, kind: str) -> np.ndarray:
    """The pq x pq filter of Sec. 5 for bases U_A [N, p, r_a], U_B [N, q, r_b]:
    'kron' = (I - P_A) (x) (I - P_B) (Eq. (25)); 'classical' =
    I - P_A (x) P_B (Eq. (24)).  [N, pq, pq]"""
    N, p, q = U_A.shape[0], U_A.shape[1], U_B.shape[1]
    PA, PB = projector(U_A), projector(U_B)
    Ip, Iq = np.eye(p), np.eye(q)
    out = np.empty((N, p * q, p * q), dtype=np.complex128)
    for i in range(N):
        if kind == "kron":
            out[i] = np.kron(Ip - PA[i], Iq - PB[i])
        elif kind == "classical":
            out[i] = np.eye(p * q) - np.kron(PA[i], PB[i])
        else:
            raise ValueError(kind)
    return out


def steering_matrix(p: int, b: np.ndarray) -> np.ndarray:
    """E = I_p (x) b (pq x p): d = E h = h (x) b."""
    return np.kron(np.eye(p), np.asarray(b, np.complex128).reshape(-1, 1))


def glrt_explicit(F: np.ndarray, Xt: np.ndarray, b: np.ndarray, h: Optional[np.ndarray] = None,
                  parts: int = 1):
    """Statistic of reading V1 for filters F [N, pq, pq], test snapshots
    Xt [N, p, q] (x = vec(X^T)) and one temporal steering b [q].  Returns
    (T [N], u [N, p]) where u = E^H F x."""
    N, p, q = Xt.shape
    b = np.asarray(b, np.complex128)
    E = steering_matrix(p, b)
    x = Xt.reshape(N, p * q)                                   # vec(X^T): x[i q + j] = X[i, j]
    Fx = np.matmul(F, x[..., None])[..., 0]
    u = np.matmul(np.conj(E.T)[None], Fx[..., None])[..., 0]   # [N, p]
    G = np.matmul(np.conj(E.T)[None], np.matmul(F, E[None]))  # [N, p, p]
    G = (G + np.conj(np.swapaxes(G, -1, -2))) / 2.0
    bb = float(np.real(np.vdot(b, b)))
    if h is None:
        lam, V = np.linalg.eigh(G)
        keep = lam > 1e-12 * bb
        inv = np.where(keep, 1.0 / np.where(keep, lam, 1.0), 0.0)
        c = np.matmul(np.conj(np.swapaxes(V, -1, -2)), u[..., None])[..., 0]
        T = np.sum(inv * np.abs(c) ** 2, axis=1)
    else:
        h = np.asarray(h, np.complex128).reshape(p)
        num = np.abs(np.matmul(np.conj(h)[None, None, :], u[..., None])[:, 0, 0]) ** 2
        den = np.real(np.einsum("i,nij,j->n", np.conj(h), G, h))
        ok = den > 1e-12 * bb * float(np.real(np.vdot(h, h)))
        T = np.where(ok, num / np.where(ok, den, 1.0), 0.0)
    return T, u


def sar_intensity(Xt: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Single-antenna matched-filter intensity |sum_k X[0, k] conj(b_k)|^2 / ||b||^2 (V3)."""
    b = np.asarray(b, np.complex128)
    s = np.sum(Xt[:, 0, :] * np.conj(b)[None, :], axis=1)
    return np.abs(s) ** 2 / float(np.real(np.vdot(b, b)))


def temporal_denominator(U_B: np.ndarray, b: np.ndarray) -> np.ndarray:
    """b^H (I - U_B U_B^H) b per pixel."""
    b = np.asarray(b, np.complex128)
    PB = projector(U_B)
    return np.real(np.vdot(b, b) - np.einsum("k,nkl,l->n", np.conj(b), PB, b))


def variant_pixels(x: np.ndarray, pixels: np.ndarray, cfg: VariantConfig, chunk: int = 256) -> dict:
    """The pass with the variant statistic on pixels [(r, c), ...].  Returns
    T, D, bin, E (enhancement), T_pass [N, K], C [N, K-1], the estimator's
    U_A, U_B, lam_A, lam_B, eta, iters, and valid."""
    p, H, W, q = x.shape
    if p != cfg.p or q != cfg.q:
        raise ValueError("frame shape does not match the configuration")
    K = cfg.passes
    if K < 1 or p % K != 0:
        raise ValueError("p must be a multiple of the number of passes")
    if K > 1 and cfg.filter != "kron":
        raise ValueError("several passes are combined with the Kron-STAP filter only")
    pp = p // K
    st = cfg.training_stencil()
    r0, r1, c0, c1 = valid_region(H, W, st)
    pixels = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    npx = pixels.shape[0]
    rows, cols = pixels[:, 0], pixels[:, 1]
    valid = (rows >= r0) & (rows < r1) & (cols >= c0) & (cols < c1)
    tau = cfg.threshold()
    bank = cfg.steering_set()
    h = None if cfg.stat_mode == "glrt" else np.asarray(cfg.h_steer, np.complex128).reshape(p)
    out = dict(T=np.zeros(npx), D=np.zeros(npx, np.uint8), bin=np.zeros(npx, np.int64), E=np.zeros(npx),
               T_pass=np.zeros((npx, K)), C=np.zeros((npx, max(K - 1, 0))),
               T_bins=np.zeros((npx, bank.shape[0])),
               U_A=np.zeros((npx, p, cfg.r_a), np.complex128), U_B=np.zeros((npx, q, cfg.r_b), np.complex128),
               lam_A=np.zeros((npx, p)), lam_B=np.zeros((npx, q)), eta=np.zeros(npx),
               iters=np.zeros(npx, np.int64), valid=valid, tau=tau)
    vidx = np.nonzero(valid)[0]
    for s0 in range(0, vidx.size, chunk):
        ids = vidx[s0:s0 + chunk]
        rr, cc = rows[ids], cols[ids]
        S = sample_covariance(x, rr, cc, st)
        Xt = snapshots(x, rr, cc)
        finite = np.isfinite(S.reshape(ids.size, -1)).all(1) & np.isfinite(Xt.reshape(ids.size, -1)).all(1)
        S = np.where(finite[:, None, None], S, 0.0)
        Xt = np.where(finite[:, None, None], Xt, 0.0)
        est = lr_kron(rearrange(S, p, q), p, q, cfg.r_a, cfg.r_b, cfg.eps, cfg.min_iter, cfg.max_iter)
        F = filter_matrix(est["U_A"], est["U_B"], cfg.filter)
        Tb = np.zeros((ids.size, bank.shape[0]))
        Tp = np.zeros((ids.size, bank.shape[0], K))
        Ib = np.zeros((ids.size, bank.shape[0]))
        for m, b in enumerate(bank):
            t, u = glrt_explicit(F, Xt, b, h)
            Tb[:, m] = t
            Ib[:, m] = sar_intensity(Xt, b)
            if K > 1:
                den = temporal_denominator(est["U_B"], b)
                ok = den > 1e-12 * float(np.real(np.vdot(b, b)))
                e2 = np.abs(u) ** 2
                for k in range(K):
                    Tp[:, m, k] = np.where(ok, e2[:, k * pp:(k + 1) * pp].sum(1) / np.where(ok, den, 1.0), 0.0)
        best = np.argmax(Tb, axis=1)
        sel = np.arange(ids.size)
        t = Tb[sel, best]
        isar = Ib[sel, best]
        enh = np.where(isar > 0.0, t / np.where(isar > 0.0, isar, 1.0), 0.0)
        zero = est["zero"]
        t = np.where(zero, 0.0, t)
        enh = np.where(zero, 0.0, enh)
        t = np.where(finite, t, np.nan)
        enh = np.where(finite, enh, np.nan)
        out["T"][ids] = t
        out["D"][ids] = (finite & (t > tau)).astype(np.uint8)
        out["bin"][ids] = best
        out["E"][ids] = enh
        out["T_bins"][ids] = np.where(zero[:, None], 0.0, Tb)
        if K > 1:
            tp = np.where(zero[:, None], 0.0, Tp[sel, best])
            tp = np.where(finite[:, None], tp, np.nan)
            out["T_pass"][ids] = tp
            out["C"][ids] = np.sqrt(tp[:, 1:]) - np.sqrt(tp[:, :1])
        else:
            out["T_pass"][ids, 0] = t
        out["U_A"][ids], out["U_B"][ids] = est["U_A"], est["U_B"]
        out["lam_A"][ids], out["lam_B"][ids] = est["lam_A"], est["lam_B"]
        out["eta"][ids], out["iters"][ids] = est["eta"], est["iters"]
    return out


def variant_frame(x: np.ndarray, cfg: VariantConfig) -> dict:
    """variant_pixels over every valid pixel, plus [H, W] images T_img, D_img,
    E_img, bin_img and [K, H, W] T_pass_img, [K-1, H, W] C_img."""
    p, H, W, q = x.shape
    st = cfg.training_stencil()
    r0, r1, c0, c1 = valid_region(H, W, st)
    rr, cc = np.meshgrid(np.arange(r0, r1), np.arange(c0, c1), indexing="ij")
    pix = np.stack([rr.ravel(), cc.ravel()], 1)
    out = variant_pixels(x, pix, cfg)
    K = cfg.passes
    imgs = dict(T_img=np.zeros((H, W)), D_img=np.zeros((H, W), np.uint8), E_img=np.zeros((H, W)),
                bin_img=np.zeros((H, W), np.int64), T_pass_img=np.zeros((K, H, W)),
                C_img=np.zeros((max(K - 1, 0), H, W)))
    r, c = pix[:, 0], pix[:, 1]
    imgs["T_img"][r, c] = out["T"]
    imgs["D_img"][r, c] = out["D"]
    imgs["E_img"][r, c] = out["E"]
    imgs["bin_img"][r, c] = out["bin"]
    for k in range(K):
        imgs["T_pass_img"][k, r, c] = out["T_pass"][:, k]
    for k in range(K - 1):
        imgs["C_img"][k, r, c] = out["C"][:, k]
    out.update(imgs)
    out["pixels"] = pix
    return out
