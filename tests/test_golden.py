"""The stored expected values under tests/golden/ (written by
tests/golden/make_golden.py from the FP64 oracle alone).

On the CPU: the scene generator still produces the fingerprinted inputs, and
the oracle still reproduces the stored outputs.  A change to the oracle's
arithmetic that moves them must regenerate the fixtures, naming the passage
of the paper that justifies it.  The GPU parity suite compares the HIP path
with the same stored values.
"""
import importlib.util
import os

import numpy as np
import pytest

import oracle
import scenegen

_spec = importlib.util.spec_from_file_location(
    "make_golden", os.path.join(os.path.dirname(__file__), "golden", "make_golden.py"))
golden = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(golden)


@pytest.mark.parametrize("name", sorted(golden.FIXTURES))
def test_golden_inputs_are_unchanged(name):
    spec, seed, base, _, _ = golden.FIXTURES[name]
    head, table = golden.read(name)
    sc = scenegen.make_scene(spec, seed=seed)
    assert head["x_sha256"] == golden.scene_sha256(sc.x)
    assert head["config"] == str(base) and int(head["seed"]) == seed
    pix = golden.fixture_pixels(spec, sc, oracle.OracleConfig(**base), golden.FIXTURES[name][3],
                                golden.FIXTURES[name][4])
    assert np.array_equal(pix[:, 0], table["r"]) and np.array_equal(pix[:, 1], table["c"])


@pytest.mark.parametrize("name", sorted(golden.FIXTURES))
def test_oracle_reproduces_golden(name):
    head, table = golden.read(name)
    _, cfg, _, out, gA, gB = golden.compute(name)
    assert float(head["tau"]) == pytest.approx(out["tau"], rel=1e-14)
    np.testing.assert_allclose(out["T"], table["T"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(out["eta"], table["eta"], rtol=1e-7, atol=1e-12)
    assert np.array_equal(out["iters"], table["iters"])
    # D is decided on T, away from the threshold
    away = np.abs(table["T"] - out["tau"]) > 1e-6 * out["tau"]
    assert np.array_equal(out["D"][away], table["D"][away])
    np.testing.assert_allclose(gA, table["gap_A"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gB, table["gap_B"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("name", sorted(golden.FIXTURES))
def test_golden_fixture_is_meaningful(name):
    """Most stored pixels are valid and graded, and some are detections."""
    head, t = golden.read(name)
    valid = t["iters"] > 0
    graded = valid & (t["gap_A"] >= 1e-3) & (t["gap_B"] >= 1e-3)
    assert graded.sum() >= 0.8 * len(t["T"]) - 6
    assert t["D"].sum() >= 1
    # outside the valid region the pass emits zeros
    assert np.all(t["T"][~valid] == 0) and np.all(t["D"][~valid] == 0)
