"""FP64 oracle of the per-pixel Kronecker STAP pass (test infrastructure only).

Per pixel (r, c) of a multichannel SAR frame x[p][H][W][q] this computes, in
complex128 and in the paper's order:

  1. the sample covariance S of the pixel's n training snapshots
     (Sec. 1.1, sample covariance matrix, Eq. (2));
  2. the rearrangement R = R(S) of Algorithm 1 (Sec. 4), p^2 x q^2;
  3. the LR-Kron alternation of Algorithm 2 (Sec. 4) giving the rank-r_a
     space factor A-hat and the time factor B-hat, truncated to rank r_b once
     at the end (the relaxation described in Sec. 4 after the definition of
     EIG_r, Eq. (17));
  4. the Kron-STAP projector F = (I - U_A U_A^H) (x) (I - U_B U_B^H)
     (Sec. 5, Eq. (25)) applied as a matched filter w = F d (Eq. (23)) and
     the pixel statistic maximised over the spatial steering h as in Sec. 6.3
     (Eq. (26)), normalised by d^H F d;
  5. the detection bit D = T > tau.

Readings taken where the paper is silent, ambiguous or garbled:

  R1  x = vec(X^T) (Sec. 2) is used, i.e. x[i*q + j] = X[i, j]; Sec. 1.1 writes
      vec(X), which is not compatible with a p x p space factor on the left of
      the Kronecker product.
  R2  The SCM is (1/n) sum x x^H (Eq. (2)); Algorithm 2 writes x x^T.
  R3  R follows Algorithm 1's orientation, under which R(A (x) B) =
      vec(A) vec(B)^T with column-major vec (as Eq. (16) requires); the prose
      before Eq. (15) would give vec(A^T) instead.
  R4  Algorithm 1's unbalanced parenthesis in L is read as
      q*(J - p*floor((J-1)/p) - 1), the only in-range reading.
  R5  The initialiser a_0 = R 1 / q^2 uses the all-ones vector of length q^2
      (R has q^2 columns); it equals the block-sum form of Eq. (19).  If
      ||a_0|| <= 1e-12 ||R||_F it falls back to a_0 = R vec(I_q) (not in the
      paper).
  R6  Loop test: |eta_k - eta_{k-1}| > eps with eta_{-1} = +inf, at least
      `min_iter` and at most `max_iter` iterations; eps <= 0 runs exactly
      `max_iter` iterations.
  R7  B-hat uses one more half-step b = R^T conj(a) / ||a||^2 from the final a
      (the least-squares time factor for the returned space factor).
  R8  EIG_r keeps the r eigenpairs of largest algebraic value of the Hermitian
      part of its argument (all iterates are PSD in exact arithmetic).
  R9  Pixel statistic: T = max_h |d^H F x|^2 / (d^H F d) with d = h (x) b_s,
      which equals ||F_A X conj(F_B b_s)||^2 / (b_s^H F_B b_s); `fixed`
      mode uses one given h instead of the maximum.  T = 0 when
      b_s^H F_B b_s <= 1e-12 ||b_s||^2.
  R10 Training stencil: window offsets [-W/2, W/2-1]^2 minus a centred
      guard x guard block, ordered by (dr^2 + dc^2, dr, dc), first n kept;
      W defaults to the smallest even value >= 10 with W^2 - guard^2 >= n.
      Only pixels whose whole stencil lies inside the frame are processed
      (T = D = 0 elsewhere).
  R11 An all-zero training set gives T = 0; any non-finite training or test
      sample gives T = NaN, D = 0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


# --------------------------------------------------------------------------
# configuration
# --------------------------------------------------------------------------
@dataclasses.dataclass
class OracleConfig:
    p: int
    q: int
    n: int
    r_a: int = 1
    r_b: int = 3
    window: int = 0
    guard: int = 3
    stencil: Optional[np.ndarray] = None   # explicit (n, 2) int (dr, dc); overrides n/window/guard
    eps: float = 1e-6
    min_iter: int = 2
    max_iter: int = 50
    stat_mode: str = "glrt"                 # "glrt" (max over h) or "fixed" (given h)
    b_steer: Optional[np.ndarray] = None    # q complex; None = ones
    h_steer: Optional[np.ndarray] = None    # p complex; fixed mode only
    tau: float = 0.0                        # > 0: used as given
    pfa: float = 1e-4                       # else tau = Gamma(p - r_a, 1) upper-tail quantile

    def training_stencil(self) -> np.ndarray:
        if self.stencil is not None:
            return np.asarray(self.stencil, dtype=np.int64).reshape(-1, 2)
        return default_stencil(self.n, self.window, self.guard)

    def threshold(self) -> float:
        if self.tau > 0:
            return float(self.tau)
        return gamma_upper_quantile(self.p - self.r_a, self.pfa)

    def temporal_steering(self) -> np.ndarray:
        if self.b_steer is None:
            return np.ones(self.q, dtype=np.complex128)
        return np.asarray(self.b_steer, dtype=np.complex128).reshape(self.q)


# --------------------------------------------------------------------------
# training stencil and valid region (reading R10)
# --------------------------------------------------------------------------
def stencil_window(n: int, guard: int = 3) -> int:
    w = 10
    while w * w - guard * guard < n:
        w += 2
    return w


def default_stencil(n: int, window: int = 0, guard: int = 3) -> np.ndarray:
    if guard < 1 or guard % 2 == 0:
        raise ValueError("guard must be odd and >= 1")
    w = window if window > 0 else stencil_window(n, guard)
    half, g = w // 2, guard // 2
    cand = [(dr, dc) for dr in range(-half, w - half) for dc in range(-half, w - half)
            if not (abs(dr) <= g and abs(dc) <= g)]
    if len(cand) < n:
        raise ValueError("window too small for n training vectors")
    cand.sort(key=lambda t: (t[0] * t[0] + t[1] * t[1], t[0], t[1]))
    return np.array(cand[:n], dtype=np.int64)


def valid_region(H: int, W: int, stencil: np.ndarray):
    """Half-open (r0, r1, c0, c1) of pixels whose whole stencil is inside."""
    dr, dc = stencil[:, 0], stencil[:, 1]
    r0 = max(0, -int(dr.min()))
    r1 = H - max(0, int(dr.max()))
    c0 = max(0, -int(dc.min()))
    c1 = W - max(0, int(dc.max()))
    return r0, max(r0, r1), c0, max(c0, c1)


# --------------------------------------------------------------------------
# snapshots and sample covariance (Sec. 1.1, Eq. (2); Sec. 2 for vec(X^T))
# --------------------------------------------------------------------------
def snapshots(x: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """X[k] = p x q snapshot of pixel (rows[k], cols[k]); complex128."""
    return np.ascontiguousarray(x[:, rows, cols, :].transpose(1, 0, 2)).astype(np.complex128)


def sample_covariance(x: np.ndarray, rows: np.ndarray, cols: np.ndarray,
                      stencil: np.ndarray) -> np.ndarray:
    """S = (1/n) sum_m x_m x_m^H over the stencil, x_m = vec(X_m^T). [N, pq, pq]"""
    p, q = x.shape[0], x.shape[3]
    n = stencil.shape[0]
    rr = rows[:, None] + stencil[None, :, 0]
    cc = cols[:, None] + stencil[None, :, 1]
    tr = x[:, rr, cc, :]                                   # [p, N, n, q]
    v = tr.transpose(1, 2, 0, 3).reshape(rows.size, n, p * q).astype(np.complex128)
    # columns of the pq x n training matrix are v[k, m, :]
    return np.matmul(v.transpose(0, 2, 1), v.conj()) / n


# --------------------------------------------------------------------------
# Algorithm 1: rearrangement operator (literal index grids, 1-based)
# --------------------------------------------------------------------------
def rearrange(S: np.ndarray, p: int, q: int) -> np.ndarray:
    """R(S) in C^{p^2 x q^2} following Algorithm 1 (reading R4)."""
    S = np.asarray(S)
    batch = S.shape[:-2]
    pq = p * q
    s = np.swapaxes(S, -1, -2).reshape(batch + (pq * pq,))       # vec(S), column-major
    P = np.arange(1, q * q + 1)[:, None] * np.ones((1, p * p), dtype=np.int64)
    J = np.ones((q * q, 1), dtype=np.int64) * np.arange(1, p * p + 1)[None, :]
    L = P - q * ((P - 1) // q) + q * (J - p * ((J - 1) // p) - 1)
    N = -(-P // q) + q * (-(-J // p) - 1)                        # ceil via negated floor
    M = L + (N - 1) * pq
    Rt = s[..., M - 1]                                           # [.., q^2, p^2]: entry (i, j) = s_{M_ij}
    return np.swapaxes(Rt, -1, -2)                               # R_{ji} = s_{M_ij}


def rearrange_direct(S: np.ndarray, p: int, q: int) -> np.ndarray:
    """Block form of the same operator: row a*p+b holds vec(S(b, a)) (0-based),
    where S(b, a) is the q x q block of Eq. (15)'s block notation."""
    S = np.asarray(S)
    batch = S.shape[:-2]
    R = np.empty(batch + (p * p, q * q), dtype=S.dtype)
    for a in range(p):
        for b in range(p):
            blk = S[..., b * q:(b + 1) * q, a * q:(a + 1) * q]
            R[..., a * p + b, :] = np.swapaxes(blk, -1, -2).reshape(batch + (q * q,))
    return R


def _vec(M: np.ndarray) -> np.ndarray:
    """Column-major vec of the last two axes."""
    return np.swapaxes(M, -1, -2).reshape(M.shape[:-2] + (M.shape[-1] * M.shape[-2],))


def _mv(M: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Batched matrix-vector product M[k] @ v[k]."""
    return np.matmul(M, v[..., None])[..., 0]


def _mtv(M: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Batched M[k]^T @ v[k] (plain transpose, no conjugation)."""
    return np.matmul(np.swapaxes(M, -1, -2), v[..., None])[..., 0]


def _unvec(v: np.ndarray, m: int) -> np.ndarray:
    return np.swapaxes(v.reshape(v.shape[:-1] + (m, m)), -1, -2)


# --------------------------------------------------------------------------
# EIG_r (Sec. 4, Eq. (17); reading R8)
# --------------------------------------------------------------------------
def top_eigvecs(M: np.ndarray, r: int):
    """Eigenpairs of the Hermitian part of M, largest algebraic value first."""
    Hm = (M + np.conj(np.swapaxes(M, -1, -2))) / 2.0
    lam, V = np.linalg.eigh(Hm)
    lam = lam[..., ::-1]
    V = V[..., ::-1]
    return lam, V[..., :r], V


def eig_truncate(M: np.ndarray, r: int):
    """EIG_r(M) = sum_{i<=r} sigma_i u_i u_i^H; returns (EIG_r(M), U_r, sigma)."""
    lam, Ur, _ = top_eigvecs(M, r)
    lr = lam[..., :r]
    E = np.matmul(Ur * lr[..., None, :], np.conj(np.swapaxes(Ur, -1, -2)))
    return E, Ur, lam


# --------------------------------------------------------------------------
# Algorithm 2: LR-Kron (batched over pixels, per-pixel stop rule R6)
# --------------------------------------------------------------------------
def lr_kron(R: np.ndarray, p: int, q: int, r_a: int, r_b: int,
            eps: float = 1e-6, min_iter: int = 2, max_iter: int = 50, truncate_b: bool = True) -> dict:
    """Algorithm 2 on R [N, p^2, q^2] (or one R).  truncate_b=False skips the
    final rank-r_b eigendecomposition of B-hat (U_B, lam_B are then None)."""
    R = np.asarray(R, dtype=np.complex128)
    single = R.ndim == 2
    if single:
        R = R[None]
    N = R.shape[0]
    Rn = np.linalg.norm(R.reshape(N, -1), axis=1)              # ||R||_F
    zero = Rn == 0.0
    Rs = np.where(zero[:, None, None], 1.0, R)                  # keep the arithmetic finite
    Rn_s = np.where(zero, 1.0, Rn)

    # initialisation a_0 = R 1_{q^2} / q^2 (reading R5)
    a = _mv(Rs, np.ones((N, q * q))) / (q * q)
    small = np.linalg.norm(a, axis=1) <= 1e-12 * Rn_s
    if np.any(small):
        a_alt = _mv(Rs, np.broadcast_to(_vec(np.eye(q)), (N, q * q)))
        a = np.where(small[:, None], a_alt, a)

    eta = np.zeros(N)
    eta_prev = np.full(N, np.inf)
    iters = np.zeros(N, dtype=np.int64)
    active = ~zero
    U_A = np.zeros((N, p, r_a), dtype=np.complex128)
    lam_A = np.zeros((N, p))
    while np.any(active):
        idx = np.nonzero(active)[0]
        Ri, ai = Rs[idx], a[idx]
        b = _mtv(Ri, np.conj(ai)) / np.sum(np.abs(ai) ** 2, 1)[:, None]      # R^T a* / ||a||^2
        an = _mv(Ri, np.conj(b)) / np.sum(np.abs(b) ** 2, 1)[:, None]       # R b* / ||b||^2
        A, Ua, lamA = eig_truncate(_unvec(an, p), r_a)
        an = _vec(A)
        resid = Ri - an[:, :, None] * b[:, None, :]
        e = np.linalg.norm(resid.reshape(idx.size, -1), axis=1) / Rn_s[idx]
        a[idx] = an
        U_A[idx] = Ua
        lam_A[idx] = lamA
        iters[idx] += 1
        k = iters[idx]
        done = (k >= max_iter) | ((k >= min_iter) & (np.abs(e - eta_prev[idx]) <= eps) & (eps > 0))
        eta[idx] = e
        eta_prev[idx] = e
        active[idx[done]] = False

    # final half-step and the single rank-r_b truncation (readings R7, R8)
    bfin = _mtv(Rs, np.conj(a)) / np.sum(np.abs(a) ** 2, 1)[:, None]
    Bm = _unvec(bfin, q)
    Bm = (Bm + np.conj(np.swapaxes(Bm, -1, -2))) / 2.0
    lam_B, U_B = (top_eigvecs(Bm, r_b)[:2]) if truncate_b else (None, None)
    Am = _unvec(a, p)
    out = dict(A=Am, B=Bm, U_A=U_A, U_B=U_B, eta=eta, iters=iters,
               lam_A=lam_A, lam_B=lam_B, zero=zero)
    if single:
        out = {k: (None if v is None else v[0]) for k, v in out.items()}
    return out


# --------------------------------------------------------------------------
# Kron-STAP statistic (Sec. 5, Eqs. (23), (25); Sec. 6.3, Eq. (26); reading R9)
# --------------------------------------------------------------------------
def kron_stap_statistic(Xt: np.ndarray, U_A: np.ndarray, U_B: np.ndarray,
                        b_s: np.ndarray, h: Optional[np.ndarray] = None) -> np.ndarray:
    """T for test snapshots Xt [N, p, q] given orthonormal U_A [N, p, r_a],
    U_B [N, q, r_b] and temporal steering b_s [q]."""
    Xt = np.asarray(Xt, dtype=np.complex128)
    single = Xt.ndim == 2
    if single:
        Xt, U_A, U_B = Xt[None], U_A[None], U_B[None]
    b_s = np.asarray(b_s, dtype=np.complex128)
    N = Xt.shape[0]
    UBh = np.conj(np.swapaxes(U_B, -1, -2))
    UAh = np.conj(np.swapaxes(U_A, -1, -2))
    bb = np.broadcast_to(b_s, (N, b_s.size))
    # g = F_B b_s
    g = bb - _mv(U_B, _mv(UBh, bb))
    # w = X_t conj(g); z = F_A w
    w = _mv(Xt, np.conj(g))
    z = w - _mv(U_A, _mv(UAh, w))
    den = np.real(np.sum(np.conj(b_s)[None, :] * g, axis=1))     # b_s^H F_B b_s
    ok = den > 1e-12 * np.real(np.vdot(b_s, b_s))
    if h is None:
        num = np.sum(np.abs(z) ** 2, axis=1)
        T = np.where(ok, num / np.where(ok, den, 1.0), 0.0)
    else:
        h = np.asarray(h, dtype=np.complex128)
        hh = np.broadcast_to(h, (N, h.size))
        fah = hh - _mv(U_A, _mv(UAh, hh))
        hfh = np.real(np.sum(np.conj(h)[None, :] * fah, axis=1))  # h^H F_A h
        ok = ok & (hfh > 1e-12 * np.real(np.vdot(h, h)))
        num = np.abs(np.sum(np.conj(h)[None, :] * z, axis=1)) ** 2
        T = np.where(ok, num / np.where(ok, den * hfh, 1.0), 0.0)
    return T[0] if single else T


# --------------------------------------------------------------------------
# CFAR threshold: under white noise and exact subspaces T ~ Gamma(p - r_a, 1)
# --------------------------------------------------------------------------
def gamma_upper_quantile(k: int, pfa: float) -> float:
    """tau with P(Gamma(k, 1) > tau) = pfa, for integer k >= 1, by bisection on
    the closed-form survival function exp(-t) sum_{i<k} t^i / i!."""
    if k < 1 or not (0.0 < pfa < 1.0):
        raise ValueError("need k >= 1 and 0 < pfa < 1")

    def sf(t):
        term, s = 1.0, 1.0
        for i in range(1, k):
            term *= t / i
            s += term
        return math.exp(-t) * s

    lo, hi = 0.0, 1.0
    while sf(hi) > pfa:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if sf(mid) > pfa:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# --------------------------------------------------------------------------
# whole pass over a list of pixels / a frame
# --------------------------------------------------------------------------
def kron_stap_pixels(x: np.ndarray, pixels: np.ndarray, cfg: OracleConfig,
                     chunk_elems: int = 1 << 23) -> dict:
    """Run the pass on pixels [(r, c), ...]; pixels outside the valid region
    get T = D = 0.  Returns T, D, U_A, U_B, eta, iters, lam_A, lam_B, valid."""
    p, H, W, q = x.shape
    if p != cfg.p or q != cfg.q:
        raise ValueError("frame shape does not match the configuration")
    st = cfg.training_stencil()
    n = st.shape[0]
    r0, r1, c0, c1 = valid_region(H, W, st)
    pixels = np.asarray(pixels, dtype=np.int64).reshape(-1, 2)
    npx = pixels.shape[0]
    rows, cols = pixels[:, 0], pixels[:, 1]
    valid = (rows >= r0) & (rows < r1) & (cols >= c0) & (cols < c1)
    tau = cfg.threshold()
    b_s = cfg.temporal_steering()
    h = None if cfg.stat_mode == "glrt" else np.asarray(cfg.h_steer, np.complex128).reshape(p)
    T = np.zeros(npx)
    D = np.zeros(npx, dtype=np.uint8)
    U_A = np.zeros((npx, p, cfg.r_a), dtype=np.complex128)
    U_B = np.zeros((npx, q, cfg.r_b), dtype=np.complex128)
    eta = np.zeros(npx)
    iters = np.zeros(npx, dtype=np.int64)
    lam_A = np.zeros((npx, p))
    lam_B = np.zeros((npx, q))
    vidx = np.nonzero(valid)[0]
    step = max(1, chunk_elems // (n * p * q))
    for s0 in range(0, vidx.size, step):
        ids = vidx[s0:s0 + step]
        rr, cc = rows[ids], cols[ids]
        S = sample_covariance(x, rr, cc, st)
        Xt = snapshots(x, rr, cc)
        finite = np.isfinite(S.reshape(ids.size, -1)).all(1) & np.isfinite(Xt.reshape(ids.size, -1)).all(1)
        S = np.where(finite[:, None, None], S, 0.0)
        Xt = np.where(finite[:, None, None], Xt, 0.0)
        R = rearrange(S, p, q)
        est = lr_kron(R, p, q, cfg.r_a, cfg.r_b, cfg.eps, cfg.min_iter, cfg.max_iter)
        t = kron_stap_statistic(Xt, est["U_A"], est["U_B"], b_s, h)
        t = np.where(est["zero"], 0.0, t)
        t = np.where(finite, t, np.nan)
        T[ids] = t
        D[ids] = (finite & (t > tau)).astype(np.uint8)
        U_A[ids], U_B[ids] = est["U_A"], est["U_B"]
        eta[ids], iters[ids] = est["eta"], est["iters"]
        lam_A[ids], lam_B[ids] = est["lam_A"], est["lam_B"]
    return dict(T=T, D=D, U_A=U_A, U_B=U_B, eta=eta, iters=iters,
                lam_A=lam_A, lam_B=lam_B, valid=valid, tau=tau)


def kron_stap_frame(x: np.ndarray, cfg: OracleConfig) -> dict:
    """Full-frame T [H, W] (float64) and D [H, W] (uint8)."""
    p, H, W, q = x.shape
    st = cfg.training_stencil()
    r0, r1, c0, c1 = valid_region(H, W, st)
    rr, cc = np.meshgrid(np.arange(r0, r1), np.arange(c0, c1), indexing="ij")
    pix = np.stack([rr.ravel(), cc.ravel()], 1)
    out = kron_stap_pixels(x, pix, cfg)
    T = np.zeros((H, W))
    D = np.zeros((H, W), dtype=np.uint8)
    T[pix[:, 0], pix[:, 1]] = out["T"]
    D[pix[:, 0], pix[:, 1]] = out["D"]
    out["T_img"], out["D_img"] = T, D
    out["pixels"] = pix
    return out


def relative_gaps(lam: np.ndarray, r: int) -> np.ndarray:
    """(lambda_r - lambda_{r+1}) / lambda_1 for eigenvalues sorted descending;
    1 where r is 0 or equals the dimension."""
    lam = np.asarray(lam)
    m = lam.shape[-1]
    if r <= 0 or r >= m:
        return np.ones(lam.shape[:-1])
    top = np.maximum(np.abs(lam[..., 0]), 1e-300)
    return (lam[..., r - 1] - lam[..., r]) / top


