"""Seeded synthetic multichannel SAR scenes with Kronecker clutter.

This module only draws random numbers in the shapes the detector consumes; it
holds none of the detector's arithmetic (no covariance estimation, no
Kronecker fitting, no projection, no statistic).  Both the FP64 oracle tests
and the GPU path read the frames it writes, so the two sides see the same
bytes.

Model (Sec. 2, SIRV clutter model; Eqs. (4)-(9) of the paper):
  * one snapshot per pixel is a p x q complex array X (p channels, q azimuth
    samples); its vector form is x = vec(X^T), i.e. x[i*q + j] = X[i, j]
    (channel-major), which is the ordering under which the clutter covariance
    is A (x) B with a p x p space factor A and a q x q time factor B;
  * clutter + noise of each pixel is an independent draw from
    CN(0, A (x) B + sigma^2 I) with sigma^2 = 1 and texture tau = 1;
  * A has rank r_a (rank 1 is the calibration-error model of Eq. (9)), B has
    rank r_b; their nonzero eigenvalues are drawn from U[0.5, 1], their
    eigenvectors are the Q factor of a complex Gaussian matrix, and B is scaled
    so that tr(A (x) B)/(p q) equals the clutter-to-noise ratio (per element);
  * optionally the factors rotate slowly over the scene: within block
    (bx, by) of `block` x `block` pixels the eigenvector bases are
    expm(j*kappa*(bx*G1 + by*G2)) @ U0 with G1, G2 random Hermitian matrices of
    unit spectral norm (one pair for A, one for B);
  * moving targets follow Eq. (8): x_t = alpha * a(theta) (x) b_s with the
    spatial steering a_i = exp(j*i*theta), theta ~ U[0, 2 pi), the temporal
    factor equal to the detector's temporal steering b_s (default all-ones),
    and |alpha|^2 = 10^(SNR/10) per element.

Layout of the returned frame: complex64 array x[p][H][W][q] (q fastest): one
H x (W*q) image per channel, pixel (r, c) owning the q consecutive samples
x[i, r, c, :] of channel i.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple, Union

import numpy as np

BASE_SEED = 16040362


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    p: int
    q: int
    H: int
    W: int
    r_a: int = 1
    r_b: int = 3
    cnr_db: float = 30.0
    snr_db: Union[float, Tuple[float, float]] = 10.0
    n_targets: int = 5
    block: Optional[int] = None      # factor rotation block size (pixels); None = one factor pair
    kappa: float = 0.2               # rotation per block (radians)
    b_steer: Optional[Tuple[complex, ...]] = None   # temporal steering of targets; None = ones


# Workload shapes of the paper's single-pass Kron-STAP (Sec. 6.3) at the sizes
# this library is measured on.  Tiny frame: oracle-checkable in seconds.
TINY = SceneSpec(p=3, q=8, H=64, W=64, r_a=1, r_b=3, n_targets=5, snr_db=10.0)
# Full frame, plain FP32 path: 2048^2 pixels, p=3, q=16, slowly rotating factors.
FULL_FRAME = SceneSpec(p=3, q=16, H=2048, W=2048, r_a=1, r_b=4, n_targets=200,
                       snr_db=(0.0, 15.0), block=256)
# Mixed-precision workload: p=5, q=24, 1024^2 pixels.
MIXED = SceneSpec(p=5, q=24, H=1024, W=1024, r_a=1, r_b=4, n_targets=200,
                  snr_db=(0.0, 15.0), block=256)


def _unitary_q(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    g = (rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))) / np.sqrt(2.0)
    qm, _ = np.linalg.qr(g)
    return qm[:, :r]


def _hermitian_unit(rng: np.random.Generator, n: int) -> np.ndarray:
    g = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    h = (g + g.conj().T) / 2.0
    return h / np.max(np.abs(np.linalg.eigvalsh(h)))


def _expm_i_herm(h: np.ndarray, t: float) -> np.ndarray:
    """expm(j*t*h) for Hermitian h, via its eigendecomposition."""
    lam, v = np.linalg.eigh(h)
    return (v * np.exp(1j * t * lam)) @ v.conj().T


@dataclasses.dataclass
class Scene:
    spec: SceneSpec
    seed: int
    x: np.ndarray                    # complex64 [p][H][W][q]
    targets: np.ndarray              # int64 [n_targets, 2] (row, col)
    target_snr_db: np.ndarray        # float64 [n_targets]
    factors: list                    # per block: (A, B) complex128


def _factor_pairs(spec: SceneSpec, rng: np.random.Generator):
    p, q = spec.p, spec.q
    ua0 = _unitary_q(rng, p, spec.r_a)
    ub0 = _unitary_q(rng, q, spec.r_b)
    la = rng.uniform(0.5, 1.0, spec.r_a)
    lb = rng.uniform(0.5, 1.0, spec.r_b)
    scale = 10.0 ** (spec.cnr_db / 10.0) * p * q / (la.sum() * lb.sum())
    lb = lb * scale
    if spec.block is None:
        nby = nbx = 1
        blk = max(spec.H, spec.W)
    else:
        blk = spec.block
        nby = -(-spec.H // blk)
        nbx = -(-spec.W // blk)
    ga1, ga2 = _hermitian_unit(rng, p), _hermitian_unit(rng, p)
    gb1, gb2 = _hermitian_unit(rng, q), _hermitian_unit(rng, q)
    pairs = {}
    for by in range(nby):
        for bx in range(nbx):
            if spec.block is None:
                ua, ub = ua0, ub0
            else:
                ua = _expm_i_herm(bx * ga1 + by * ga2, spec.kappa) @ ua0
                ub = _expm_i_herm(bx * gb1 + by * gb2, spec.kappa) @ ub0
            a = (ua * la) @ ua.conj().T
            b = (ub * lb) @ ub.conj().T
            pairs[(by, bx)] = (a, b)
    return pairs, blk, nby, nbx


def make_scene(spec: SceneSpec, seed: int = BASE_SEED) -> Scene:
    """Draw one frame.  Deterministic in (spec, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p, q, H, W = spec.p, spec.q, spec.H, spec.W
    pq = p * q
    pairs, blk, nby, nbx = _factor_pairs(spec, rng)
    x = np.empty((p, H, W, q), dtype=np.complex64)
    factors = []
    for by in range(nby):
        for bx in range(nbx):
            a, b = pairs[(by, bx)]
            factors.append((a, b))
            cov = np.kron(a, b) + np.eye(pq)
            lam, v = np.linalg.eigh(cov)
            root = (v * np.sqrt(np.clip(lam, 0.0, None))) @ v.conj().T   # Hermitian square root
            r0, r1 = by * blk, min(H, (by + 1) * blk)
            c0, c1 = bx * blk, min(W, (bx + 1) * blk)
            npx = (r1 - r0) * (c1 - c0)
            w = np.empty((npx, pq), dtype=np.complex64)
            w.real = rng.standard_normal((npx, pq), dtype=np.float32)
            w.imag = rng.standard_normal((npx, pq), dtype=np.float32)
            w *= np.float32(1.0 / np.sqrt(2.0))
            snap = w @ root.T.astype(np.complex64)          # rows: root @ w_i
            snap = snap.reshape(r1 - r0, c1 - c0, p, q)
            x[:, r0:r1, c0:c1, :] = snap.transpose(2, 0, 1, 3)
    # moving targets, Eq. (8)
    nt = spec.n_targets
    rows = rng.integers(0, H, nt)
    cols = rng.integers(0, W, nt)
    if isinstance(spec.snr_db, tuple):
        snr = rng.uniform(spec.snr_db[0], spec.snr_db[1], nt)
    else:
        snr = np.full(nt, float(spec.snr_db))
    theta = rng.uniform(0.0, 2.0 * np.pi, nt)
    phase = rng.uniform(0.0, 2.0 * np.pi, nt)
    bs = np.ones(q, dtype=np.complex128) if spec.b_steer is None else np.asarray(spec.b_steer, np.complex128)
    for t in range(nt):
        alpha = np.sqrt(10.0 ** (snr[t] / 10.0)) * np.exp(1j * phase[t])
        av = np.exp(1j * theta[t] * np.arange(p))
        x[:, rows[t], cols[t], :] += (alpha * np.outer(av, bs)).astype(np.complex64)
    return Scene(spec=spec, seed=seed, x=x, targets=np.stack([rows, cols], 1),
                 target_snr_db=snr, factors=factors)


def random_pixels(H: int, W: int, count: int, seed: int,
                  region: Optional[Sequence[int]] = None) -> np.ndarray:
    """Seeded (row, col) sample of pixels, int32 [count, 2], inside
    region = (r0, r1, c0, c1) (half-open) if given."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r0, r1, c0, c1 = (0, H, 0, W) if region is None else region
    rr = rng.integers(r0, r1, count)
    cc = rng.integers(c0, c1, count)
    return np.stack([rr, cc], 1).astype(np.int32)


def white_noise(shape, seed: int) -> np.ndarray:
    """Seeded CN(0, 1) samples, complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def make_scene_torch(spec: SceneSpec, seed: int = BASE_SEED, device="cuda"):
    """The same scene model drawn on a device with torch (for large benchmark
    workloads): factor pairs and targets from NumPy's PCG64 as in make_scene,
    per-pixel Gaussian draws from a seeded torch generator on `device`.
    Returns a complex64 torch tensor [p][H][W][q] (different draws than
    make_scene for the same seed)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    p, q, H, W = spec.p, spec.q, spec.H, spec.W
    pq = p * q
    pairs, blk, nby, nbx = _factor_pairs(spec, rng)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    x = torch.empty((p, H, W, q), dtype=torch.complex64, device=device)
    for by in range(nby):
        for bx in range(nbx):
            a, b = pairs[(by, bx)]
            cov = np.kron(a, b) + np.eye(pq)
            lam, v = np.linalg.eigh(cov)
            root = (v * np.sqrt(np.clip(lam, 0.0, None))) @ v.conj().T
            r0, r1 = by * blk, min(H, (by + 1) * blk)
            c0, c1 = bx * blk, min(W, (bx + 1) * blk)
            npx = (r1 - r0) * (c1 - c0)
            w = torch.complex(torch.randn((npx, pq), generator=gen, device=device),
                              torch.randn((npx, pq), generator=gen, device=device)) * (1.0 / np.sqrt(2.0))
            rt = torch.from_numpy(root.T.astype(np.complex64)).to(device)
            snap = (w @ rt).reshape(r1 - r0, c1 - c0, p, q)
            x[:, r0:r1, c0:c1, :] = snap.permute(2, 0, 1, 3)
    nt = spec.n_targets
    rows = rng.integers(0, H, nt)
    cols = rng.integers(0, W, nt)
    snr = rng.uniform(*spec.snr_db, nt) if isinstance(spec.snr_db, tuple) else np.full(nt, float(spec.snr_db))
    theta = rng.uniform(0.0, 2.0 * np.pi, nt)
    phase = rng.uniform(0.0, 2.0 * np.pi, nt)
    bs = np.ones(q, dtype=np.complex128) if spec.b_steer is None else np.asarray(spec.b_steer, np.complex128)
    for t in range(nt):
        alpha = np.sqrt(10.0 ** (snr[t] / 10.0)) * np.exp(1j * phase[t])
        tgt = alpha * np.outer(np.exp(1j * theta[t] * np.arange(p)), bs)
        x[:, rows[t], cols[t], :] += torch.from_numpy(tgt.astype(np.complex64)).to(device)
    return x


def batch_tile_specs(seed: int = BASE_SEED + 3, ntiles: int = 64):
    """Uneven tiles: side in {128, 256, 512, 1024}, q in {8, 12, 16},
    n in {64, 128, 256}, p = 3, rank(A) in {1, 2}, rank(B) in {2..6};
    targets = max(1, round(area * 200 / 2048^2)).  Returns a list of
    (SceneSpec, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(ntiles):
        side = int(rng.choice([128, 256, 512, 1024]))
        q = int(rng.choice([8, 12, 16]))
        n = int(rng.choice([64, 128, 256]))
        ra = int(rng.integers(1, 3))
        rb = int(rng.integers(2, 7))
        nt = max(1, int(round(side * side * 200 / 2048 ** 2)))
        out.append((SceneSpec(p=3, q=q, H=side, W=side, r_a=ra, r_b=rb, n_targets=nt, snr_db=(0.0, 15.0)), n))
    return out


def serving_trace(seed: int = BASE_SEED + 4, nframes: int = 300):
    """Frame requests: square side ~ U{256..2048}, q in {8, 16},
    n ~ U{64..256}, p = 3, rank(A) = 1, rank(B) = 3, targets at 200 per
    2048^2 pixels.  Returns a list of (SceneSpec, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nframes):
        side = int(rng.integers(256, 2049))
        q = int(rng.choice([8, 16]))
        n = int(rng.integers(64, 257))
        nt = max(1, int(round(side * side * 200 / 2048 ** 2)))
        out.append((SceneSpec(p=3, q=q, H=side, W=side, r_a=1, r_b=3, n_targets=nt, snr_db=(0.0, 15.0)), n))
    return out


# ---------------------------------------------------------------- multipass
@dataclasses.dataclass(frozen=True)
class MultipassSpec:
    """K registered passes over one scene (Sec. 3): every pass sees the same
    time factor B, its own rank-one space factor u_k u_k^H, and clutter
    coefficients that correlate across passes with `coherence`."""
    passes: int
    p: int                           # channels per pass
    q: int
    H: int
    W: int
    r_b: int = 3
    coherence: float = 0.9           # correlation of the clutter coefficient between any two passes
    cnr_db: float = 30.0
    snr_db: Union[float, Tuple[float, float]] = (5.0, 15.0)
    n_targets: int = 4               # movers per pass, at independent positions


@dataclasses.dataclass
class MultipassScene:
    spec: MultipassSpec
    seed: int
    x: np.ndarray                    # complex64 [K*p][H][W][q], pass k in channels k*p .. k*p + p - 1
    targets: np.ndarray              # int64 [K * n_targets, 3] (pass, row, col)
    U_tilde: np.ndarray              # [K*p, K] orthonormal: pass k's spatial factor in block k of column k
    A_tilde: np.ndarray              # [K*p, K*p]
    B: np.ndarray                    # [q, q]


def multipass_factors(spec: MultipassSpec, rng: np.random.Generator):
    """(A_tilde, B, U_tilde) of the K-pass clutter model: A_tilde =
    U_tilde Cc U_tilde^H with U_tilde = blockdiag(u_1, ..., u_K) and
    Cc = coherence * 1 1^T + (1 - coherence) I, B of rank r_b; scaled so that
    tr(A_tilde (x) B) / (K p q) = 10^(CNR/10)."""
    K, p, q = spec.passes, spec.p, spec.q
    U = np.zeros((K * p, K), dtype=np.complex128)
    for k in range(K):
        U[k * p:(k + 1) * p, k] = _unitary_q(rng, p, 1)[:, 0]
    Cc = spec.coherence * np.ones((K, K)) + (1.0 - spec.coherence) * np.eye(K)
    A = U @ Cc @ U.conj().T
    ub = _unitary_q(rng, q, spec.r_b)
    lb = rng.uniform(0.5, 1.0, spec.r_b)
    B = (ub * lb) @ ub.conj().T
    B *= 10.0 ** (spec.cnr_db / 10.0) * K * p * q / (np.real(np.trace(A)) * np.real(np.trace(B)))
    return A, B, U


def make_multipass_scene(spec: MultipassSpec, seed: int = BASE_SEED) -> MultipassScene:
    """Draw one stacked K-pass frame: per pixel CN(0, A_tilde (x) B + I), then
    movers in single passes (Eq. (8) on that pass's channels)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    K, p, q, H, W = spec.passes, spec.p, spec.q, spec.H, spec.W
    P = K * p
    A, B, U = multipass_factors(spec, rng)
    cov = np.kron(A, B) + np.eye(P * q)
    lam, v = np.linalg.eigh(cov)
    root = (v * np.sqrt(np.clip(lam, 0.0, None))) @ v.conj().T
    npx = H * W
    w = np.empty((npx, P * q), dtype=np.complex64)
    w.real = rng.standard_normal((npx, P * q), dtype=np.float32)
    w.imag = rng.standard_normal((npx, P * q), dtype=np.float32)
    w *= np.float32(1.0 / np.sqrt(2.0))
    snap = (w @ root.T.astype(np.complex64)).reshape(H, W, P, q)
    x = np.ascontiguousarray(snap.transpose(2, 0, 1, 3))
    nt = spec.n_targets
    tg = []
    for k in range(K):
        rows = rng.integers(0, H, nt)
        cols = rng.integers(0, W, nt)
        snr = rng.uniform(*spec.snr_db, nt) if isinstance(spec.snr_db, tuple) else np.full(nt, float(spec.snr_db))
        theta = rng.uniform(0.0, 2.0 * np.pi, nt)
        phase = rng.uniform(0.0, 2.0 * np.pi, nt)
        for t in range(nt):
            alpha = np.sqrt(10.0 ** (snr[t] / 10.0)) * np.exp(1j * phase[t])
            av = np.exp(1j * theta[t] * np.arange(p))
            x[k * p:(k + 1) * p, rows[t], cols[t], :] += (alpha * np.outer(av, np.ones(q))).astype(np.complex64)
            tg.append((k, rows[t], cols[t]))
    return MultipassScene(spec=spec, seed=seed, x=x, targets=np.array(tg, dtype=np.int64).reshape(-1, 3),
                          U_tilde=U, A_tilde=A, B=B)


# ------------------------------------------------- one large covariance
def large_q_snapshots(p: int, q: int, n: int, r_a: int = 1, cnr_db: float = 30.0,
                      seed: int = BASE_SEED) -> np.ndarray:
    """Training snapshots of the paper's timing workload (Sec. 6.1): a random
    complex rank-r_a space factor A, the identity time factor B = I_q, n
    snapshots X_m (p x q) drawn from CN(0, A (x) I_q + I) with tr(A)/p =
    10^(CNR/10).  Returns complex64 [n, p, q]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ua = _unitary_q(rng, p, r_a)
    la = rng.uniform(0.5, 1.0, r_a)
    la *= 10.0 ** (cnr_db / 10.0) * p / la.sum()
    root_a = ua * np.sqrt(la)                       # A = root_a root_a^H
    w = (rng.standard_normal((n, r_a, q)) + 1j * rng.standard_normal((n, r_a, q))) / np.sqrt(2.0)
    noise = (rng.standard_normal((n, p, q)) + 1j * rng.standard_normal((n, p, q))) / np.sqrt(2.0)
    X = np.matmul(root_a[None], w) + noise          # rows of A^(1/2) W have covariance A (x) I
    return X.astype(np.complex64)


# ------------------------------------------------ SIRV texture, robustness
@dataclasses.dataclass(frozen=True)
class SirvSpec:
    """Clutter with random texture (Sec. 2, Eq. (4)): per pixel
    x = tau * c + noise with speckle c ~ CN(0, A (x) B), noise ~ CN(0, I) and
    texture tau^2 ~ Gamma(shape nu, scale 1/nu), so E[tau^2] = 1 and the
    clutter amplitude is K-distributed (texture_nu = None: tau = 1).  A has
    rank r_a, B rank r_b, scaled to E[tau^2] tr(A (x) B) / (p q) = 10^(CNR/10).

    Robustness setting: `n_test` test pixels (seeded, at least `margin` from
    the border) carry no target; around each, `n_corrupt` moving targets
    alpha a(theta) (x) b(f) (Eq. (8); a_i = exp(j i theta),
    b_k = exp(2 pi j f k)) are added at distinct offsets with Chebyshev
    distance in [inner, radius], i.e. inside the pixel's training window."""
    p: int = 3
    q: int = 16
    H: int = 96
    W: int = 96
    r_a: int = 1
    r_b: int = 3
    cnr_db: float = 30.0
    texture_nu: Optional[float] = 0.5
    n_test: int = 64
    margin: int = 16
    n_corrupt: int = 0
    radius: int = 7
    inner: int = 2
    corrupt_snr_db: float = 20.0
    corrupt_theta: float = 1.0
    corrupt_f: float = 0.25


@dataclasses.dataclass
class SirvScene:
    spec: SirvSpec
    seed: int
    x: np.ndarray                    # complex64 [p][H][W][q]
    tau2: np.ndarray                 # float64 [H][W]: the texture power of each pixel
    test_pixels: np.ndarray          # int32 [n_test, 2]
    corrupt: np.ndarray              # int64 [n_test * n_corrupt, 2]
    UA: np.ndarray                   # [p, r_a] orthonormal; A = UA diag(lamA) UA^H
    lamA: np.ndarray
    UB: np.ndarray                   # [q, r_b] orthonormal; B = UB diag(lamB) UB^H
    lamB: np.ndarray
    sigma2: float = 1.0              # noise power
    tau2_mean: float = 1.0           # E[tau^2]


def spatial_steering(p: int, theta: float) -> np.ndarray:
    """a(theta)_i = exp(j i theta), i = 0..p-1 (Eq. (8))."""
    return np.exp(1j * theta * np.arange(p))


def doppler_steering(q: int, f: float) -> np.ndarray:
    """b(f)_k = exp(2 pi j f k), k = 0..q-1: a constant Doppler shift f
    (cycles per sample) over the q samples."""
    return np.exp(2j * np.pi * f * np.arange(q))


def make_sirv_scene(spec: SirvSpec, seed: int = BASE_SEED) -> SirvScene:
    """Draw one SIRV frame with optional training-window corruption.
    Deterministic in (spec, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p, q, H, W = spec.p, spec.q, spec.H, spec.W
    ua = _unitary_q(rng, p, spec.r_a)
    ub = _unitary_q(rng, q, spec.r_b)
    la = rng.uniform(0.5, 1.0, spec.r_a)
    lb = rng.uniform(0.5, 1.0, spec.r_b)
    lb = lb * (10.0 ** (spec.cnr_db / 10.0) * p * q / (la.sum() * lb.sum()))
    root = np.kron(ua * np.sqrt(la), ub * np.sqrt(lb))              # [pq, r_a r_b]: A (x) B = root root^H
    npx = H * W
    rk = root.shape[1]
    w = (rng.standard_normal((npx, rk)) + 1j * rng.standard_normal((npx, rk))) / np.sqrt(2.0)
    noise = (rng.standard_normal((npx, p * q)) + 1j * rng.standard_normal((npx, p * q))) / np.sqrt(2.0)
    if spec.texture_nu is None:
        tau2 = np.ones(npx)
    else:
        tau2 = rng.gamma(spec.texture_nu, 1.0 / spec.texture_nu, npx)
    snap = np.sqrt(tau2)[:, None] * (w @ root.T) + noise
    x = np.ascontiguousarray(snap.reshape(H, W, p, q).transpose(2, 0, 1, 3)).astype(np.complex64)
    m = spec.margin
    tr = rng.integers(m, H - m, spec.n_test)
    tc = rng.integers(m, W - m, spec.n_test)
    offs = [(dr, dc) for dr in range(-spec.radius, spec.radius + 1) for dc in range(-spec.radius, spec.radius + 1)
            if max(abs(dr), abs(dc)) >= spec.inner]
    corrupt = []
    if spec.n_corrupt > 0:
        d = np.kron(spatial_steering(p, spec.corrupt_theta), doppler_steering(q, spec.corrupt_f))
        amp = np.sqrt(10.0 ** (spec.corrupt_snr_db / 10.0))
        for t in range(spec.n_test):
            pick = rng.choice(len(offs), spec.n_corrupt, replace=False)
            for k in pick:
                r, c = tr[t] + offs[k][0], tc[t] + offs[k][1]
                phase = rng.uniform(0.0, 2.0 * np.pi)
                x[:, r, c, :] += (amp * np.exp(1j * phase) * d).reshape(p, q).astype(np.complex64)
                corrupt.append((r, c))
    return SirvScene(spec=spec, seed=seed, x=x, tau2=tau2.reshape(H, W), test_pixels=np.stack([tr, tc], 1).astype(np.int32),
                     corrupt=np.array(corrupt, dtype=np.int64).reshape(-1, 2), UA=ua, lamA=la, UB=ub, lamB=lb)
