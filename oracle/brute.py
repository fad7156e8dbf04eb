"""Exhaustive enumeration over all interpretations (O5), for programs of at most
16 atoms. Test infrastructure only.

* Least model: a definite program's least model is the intersection of all
  of its models (model-intersection property, Section 2.1: "I is the least
  model if I is a subset of every model J").
* Stable models: I is stable iff I = LM(P^I), P^I the Gelfond-Lifschitz
  reduct. P^I depends only on which negated atoms are in I, so every subset
  s of the negated atoms Q gives one reduct P^s; the stable models are the
  LM(P^s) with LM(P^s) and Q meeting exactly in s.

Interpretations are integers: bit a set iff atom a is true.
"""
from __future__ import annotations

import numpy as np


def _masks(prog):
    rules = []
    for h, body in prog.rules():
        pos = 0
        negm = 0
        for lit in body:
            if lit >= 0:
                pos |= 1 << lit
            else:
                negm |= 1 << (-lit - 1)
        rules.append((h, pos, negm))
    return rules


def _lm_of(rules_pos, n_atoms):
    """Intersection of all models of the definite rules [(head, posmask)]."""
    allI = np.arange(1 << n_atoms, dtype=np.int64)
    ok = np.ones(allI.shape[0], dtype=bool)
    for h, pos in rules_pos:
        ok &= ((allI & pos) != pos) | (((allI >> h) & 1) == 1)
    return int(np.bitwise_and.reduce(allI[ok])) if n_atoms else 0


def least_model(prog) -> int:
    assert prog.n_atoms <= 16
    rules = _masks(prog)
    assert all(negm == 0 for _, _, negm in rules), "definite programs only"
    return _lm_of([(h, pos) for h, pos, _ in rules], prog.n_atoms)


def stable_models(prog) -> list[int]:
    """All stable models as sorted interpretation integers."""
    assert prog.n_atoms <= 16
    rules = _masks(prog)
    qmask = 0
    for _, _, negm in rules:
        qmask |= negm
    qs = [a for a in range(prog.n_atoms) if (qmask >> a) & 1]
    out = set()
    for sub in range(1 << len(qs)):
        s = 0
        for t, q in enumerate(qs):
            if (sub >> t) & 1:
                s |= 1 << q
        reduct = [(h, pos) for h, pos, negm in rules if (negm & s) == 0]
        lm = _lm_of(reduct, prog.n_atoms)
        if (lm & qmask) == s:
            out.add(lm)
    return sorted(out)


def to_vector(interp: int, n_atoms: int) -> np.ndarray:
    return np.array([(interp >> a) & 1 for a in range(n_atoms)], dtype=np.uint8)


def from_vector(v) -> int:
    return sum(1 << a for a, x in enumerate(v) if x)
