"""Writes the stored expected values under tests/golden/ from the FP64 oracle.

Run from the repository root:  python tests/golden/make_golden.py

Each fixture is a seeded synthetic scene (scenegen: the input draws only) and
a set of pixels with the oracle's outputs there: the Kron-STAP statistic T of
Eq. (25) under the spatial-steering GLRT of Sec. 6.3, the detection bit
D = [T > tau], the LR-Kron fit's final residual eta and iteration count
(Algorithm 2), and the truncation gaps (lambda_r - lambda_{r+1}) / lambda_1 of
both factors, which decide whether a pixel's subspaces are unique enough to
grade.  The scene's bytes are fingerprinted so a change of the generator is
caught before any value is compared.  Only the oracle computes what is stored.
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import scenegen  # noqa: E402

# name -> (scene spec, seed, oracle configuration, random pixel count, pixel seed)
FIXTURES = {
    "tiny_frame_p3q8n64": (scenegen.TINY, scenegen.BASE_SEED,
                           dict(p=3, q=8, n=64, r_a=1, r_b=3), 31, 21),
    "frame96_p3q16n200": (scenegen.SceneSpec(p=3, q=16, H=96, W=96, r_a=1, r_b=4, n_targets=6,
                                             snr_db=(0.0, 15.0), block=32),
                          scenegen.BASE_SEED + 70, dict(p=3, q=16, n=200, r_a=1, r_b=4), 34, 22),
}

COLUMNS = ("r", "c", "T", "D", "eta", "iters", "gap_A", "gap_B")


def scene_sha256(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()


def fixture_pixels(spec, scene, cfg, count, pix_seed):
    """The scene's targets, the four corners of the valid region and a seeded
    sample of valid pixels."""
    r0, r1, c0, c1 = oracle.valid_region(spec.H, spec.W, cfg.training_stencil())
    corners = np.array([[r0, c0], [r0, c1 - 1], [r1 - 1, c0], [r1 - 1, c1 - 1]], np.int64)
    rnd = scenegen.random_pixels(spec.H, spec.W, count, pix_seed, region=(r0, r1, c0, c1))
    return np.concatenate([np.asarray(scene.targets, np.int64).reshape(-1, 2), corners,
                           rnd.astype(np.int64)])


def compute(name):
    spec, seed, base, count, pix_seed = FIXTURES[name]
    scene = scenegen.make_scene(spec, seed=seed)
    cfg = oracle.OracleConfig(**base)
    pix = fixture_pixels(spec, scene, cfg, count, pix_seed)
    out = oracle.kron_stap_pixels(scene.x, pix, cfg)
    gA = oracle.relative_gaps(out["lam_A"], cfg.r_a)
    gB = oracle.relative_gaps(out["lam_B"], cfg.r_b)
    return scene, cfg, pix, out, gA, gB


def write(name):
    spec, seed, base, _, _ = FIXTURES[name]
    scene, cfg, pix, out, gA, gB = compute(name)
    path = os.path.join(HERE, name + ".txt")
    with open(path, "w") as f:
        f.write("# Oracle outputs at sampled pixels of a seeded synthetic scene.\n")
        f.write("# T: Kron-STAP statistic, Eq. (25), maximised over the spatial steering (Sec. 6.3);\n")
        f.write("# eta, iters: LR-Kron residual and iterations (Algorithm 2); gaps: truncation gaps.\n")
        f.write("# written by: python tests/golden/make_golden.py\n")
        f.write(f"scene: {spec}\n")
        f.write(f"seed: {seed}\n")
        f.write(f"config: {base}\n")
        f.write(f"tau: {float(out['tau'])!r}\n")
        f.write(f"x_sha256: {scene_sha256(scene.x)}\n")
        f.write(" ".join(COLUMNS) + "\n")
        for i in range(pix.shape[0]):
            f.write(f"{pix[i, 0]} {pix[i, 1]} {float(out['T'][i])!r} {int(out['D'][i])} "
                    f"{float(out['eta'][i])!r} {int(out['iters'][i])} {float(gA[i])!r} {float(gB[i])!r}\n")
    return path


def read(name):
    """(header dict of strings, table dict of numpy columns) of a fixture."""
    head, rows = {}, []
    with open(os.path.join(HERE, name + ".txt")) as f:
        lines = [ln.rstrip("\n") for ln in f if not ln.startswith("#")]
    i = 0
    while lines[i].split()[0] != COLUMNS[0]:
        k, v = lines[i].split(": ", 1)
        head[k] = v
        i += 1
    for ln in lines[i + 1:]:
        rows.append([float(t) for t in ln.split()])
    a = np.array(rows)
    table = {c: a[:, j] for j, c in enumerate(COLUMNS)}
    for c in ("r", "c", "D", "iters"):
        table[c] = table[c].astype(np.int64)
    return head, table


if __name__ == "__main__":
    for nm in FIXTURES:
        print(write(nm))
