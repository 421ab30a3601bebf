"""Planted mistakes in a copy of the variant oracle (`oracle/variants.py`)
must each fail at least one pin of test_oracle_variants.py.  The mutants are
made on the CPU from the source text; the real module is never modified.
"""
import inspect
import os
import sys
import types

import pytest

from oracle import variants as V
from tests import test_oracle_variants as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "variants.py")

MUTANTS = {
    "classical filter adds the joint projector": ("out[i] = np.eye(p * q) - np.kron(PA[i], PB[i])",
                                                  "out[i] = np.eye(p * q) + np.kron(PA[i], PB[i])"),
    "Kron-STAP filter with a transposed time projector": ("out[i] = np.kron(Ip - PA[i], Iq - PB[i])",
                                                          "out[i] = np.kron(Ip - PA[i], Iq - PB[i].T)"),
    "Doppler bank of the opposite sign": ("return np.exp(2j * np.pi * (((m[:, None] * k[None, :]) % M) / M))",
                                          "return np.exp(-2j * np.pi * (((m[:, None] * k[None, :]) % M) / M))"),
    "SAR image without the conjugate steering": ("s = np.sum(Xt[:, 0, :] * np.conj(b)[None, :], axis=1)",
                                                 "s = np.sum(Xt[:, 0, :] * b[None, :], axis=1)"),
    "SAR image of channel 1": ("s = np.sum(Xt[:, 0, :] * np.conj(b)[None, :], axis=1)",
                               "s = np.sum(Xt[:, 1, :] * np.conj(b)[None, :], axis=1)"),
    "steering matrix b (x) I": ("return np.kron(np.eye(p), np.asarray(b, np.complex128).reshape(-1, 1))",
                                "return np.kron(np.asarray(b, np.complex128).reshape(-1, 1), np.eye(p))"),
    "pseudo-inverse keeps the null space": ("keep = lam > 1e-12 * bb", "keep = lam > -1.0"),
    "pass blocks overlap": ("e2[:, k * pp:(k + 1) * pp].sum(1)", "e2[:, k:k + pp].sum(1)"),
    "classical threshold with p - r_a degrees": ('dof = self.p if self.filter == "classical" else self.p - self.r_a',
                                                 "dof = self.p - self.r_a"),
    "bank keeps the smallest bin": ("best = np.argmax(Tb, axis=1)", "best = np.argmin(Tb, axis=1)"),
    "enhancement over the wrong bin": ("isar = Ib[sel, best]", "isar = Ib[sel, 0]"),
}


def _load_mutant(old, new):
    src = open(SRC).read()
    assert old in src, old
    mod = types.ModuleType("oracle.variants_mutant")
    mod.__file__ = SRC
    mod.__package__ = "oracle"
    sys.modules["oracle.variants_mutant"] = mod   # dataclasses look the module up
    try:
        exec(compile(src.replace(old, new), SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules["oracle.variants_mutant"]
    return mod


def _pin_cases():
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        marks = getattr(fn, "pytestmark", [])
        params = [m for m in marks if m.name == "parametrize"]
        if not params:
            yield fn, {}
            continue
        cases = [{}]
        for mk in params:
            argnames, values = mk.args
            names = [a.strip() for a in argnames.split(",")]
            nxt = []
            for v in values:
                v = v if isinstance(v, tuple) else (v,)
                for c in cases:
                    nxt.append(dict(c, **dict(zip(names, v))))
            cases = nxt
        for c in cases:
            yield fn, c


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_variant_mutant_fails_a_pin(mutant, monkeypatch):
    mod = _load_mutant(*MUTANTS[mutant])
    for attr, val in list(vars(mod).items()):
        if not attr.startswith("__") and hasattr(V, attr) and callable(val):
            monkeypatch.setattr(V, attr, val)
    caught = []
    for fn, kw in _pin_cases():
        try:
            fn(**kw)
        except Exception as e:  # noqa: BLE001 - any failure counts
            caught.append((fn.__name__, type(e).__name__))
    assert caught, f"no pin caught the planted mistake: {mutant}"
