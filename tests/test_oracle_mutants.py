"""Planted mistakes in a copy of the oracle must each fail at least one pin.

The mutants are made on the CPU from the oracle's source text; the real
oracle is never modified.  This shows that the pins in test_oracle_pins.py
fix the oracle's arithmetic, not only its interface.
"""
import inspect
import os
import sys
import types

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "kron_stap.py")

MUTANTS = {
    "dropped conjugate in the B half-step": ("b = _mtv(Ri, np.conj(ai))", "b = _mtv(Ri, ai)"),
    "dropped conjugate in the A half-step": ("an = _mv(Ri, np.conj(b))", "an = _mv(Ri, b)"),
    "row-major inverse vec": ("return np.swapaxes(v.reshape(v.shape[:-1] + (m, m)), -1, -2)",
                              "return v.reshape(v.shape[:-1] + (m, m))"),
    "no conjugate on the filtered steering": ("w = _mv(Xt, np.conj(g))", "w = _mv(Xt, g)"),
    "wrong sign in the spatial projector": ("z = w - _mv(U_A, _mv(UAh, w))", "z = w + _mv(U_A, _mv(UAh, w))"),
    "x x^T instead of x x^H": ("return np.matmul(v.transpose(0, 2, 1), v.conj()) / n",
                               "return np.matmul(v.transpose(0, 2, 1), v) / n"),
    "Algorithm 1 parenthesis": ("q * (J - p * ((J - 1) // p) - 1)", "q * (J - p * ((J - 1) // p))"),
    "ascending eigen order": ("    lam = lam[..., ::-1]\n    V = V[..., ::-1]\n", "    pass\n"),
    "final half-step without conjugate": ("bfin = _mtv(Rs, np.conj(a))", "bfin = _mtv(Rs, a)"),
    "truncation gap one rank late": ("return (lam[..., r - 1] - lam[..., r]) / top",
                                     "return (lam[..., r] - lam[..., min(r + 1, m - 1)]) / top"),
    "truncation gap over the smaller eigenvalue": ("return (lam[..., r - 1] - lam[..., r]) / top",
                                                   "return (lam[..., r - 1] - lam[..., r]) / lam[..., r - 1]"),
    "truncation gap without its rank-0 branch": ("if r <= 0 or r >= m:", "if r >= m:"),
}


def _load_mutant(old, new):
    src = open(SRC).read()
    assert old in src
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = SRC
    sys.modules["oracle_mutant"] = mod          # dataclasses look the module up
    try:
        exec(compile(src.replace(old, new), SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle_mutant"]
    return mod


def _pin_cases():
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_") or name == "test_p11_eigensolver_against_high_precision":
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if not params:
            yield fn, {}
            continue
        argnames, values = params[0].args
        names = [a.strip() for a in argnames.split(",")]
        for v in values:
            v = v if isinstance(v, tuple) else (v,)
            yield fn, dict(zip(names, v))


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_fails_a_pin(mutant, monkeypatch):
    mod = _load_mutant(*MUTANTS[mutant])
    for attr in oracle.__dict__:
        if hasattr(mod, attr) and callable(getattr(mod, attr)):
            monkeypatch.setattr(oracle, attr, getattr(mod, attr))
    monkeypatch.setattr(pins, "_unvec", mod._unvec)
    monkeypatch.setattr(pins, "_vec", mod._vec)
    caught = []
    for fn, kw in _pin_cases():
        try:
            fn(**kw)
        except (AssertionError, Exception) as e:  # noqa: B014 - any failure counts
            caught.append((fn.__name__, type(e).__name__))
    assert caught, f"no pin caught the planted mistake: {mutant}"
