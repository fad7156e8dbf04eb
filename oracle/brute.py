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


def sync_products(prog, guess: int = 0) -> int:
    """Number of theta(M v) evaluations of the synchronous loop (Algorithm 1,
    or one column of Algorithm 2) on the standardized positive form of
    `prog`, counting the last evaluation that changes nothing.

    Written straight from the row semantics of the standardized matrix
    (Definitions 1, 2, 5 and 7), with no matrix and no stage bookkeeping:
    a head with one rule is an AND row over that rule's body; a head with
    k >= 2 rules is an OR row over k new atoms, one AND row per rule (a
    fact among them makes its new atom a fact). For a normal program, bit t
    of `guess` is the initial value of the new atom standing for "not q_t"
    (q_t the t-th smallest negated atom), which is otherwise never derived.
    Sets are integers over atoms, and a second integer holds the new atoms
    (bit = rule index).
    """
    rules = _masks(prog)
    qmask = 0
    for _, _, negm in rules:
        qmask |= negm
    qs = [a for a in range(prog.n_atoms) if (qmask >> a) & 1]
    qbar = {q: t for t, q in enumerate(qs)}  # q -> t; "not q" reads bit t of the guess column
    by_head = {}
    for r, (h, _, _) in enumerate(rules):
        by_head.setdefault(h, []).append(r)

    def body_true(r, atoms, gbits):
        _, pos, negm = rules[r]
        if (atoms & pos) != pos:
            return False
        return all((gbits >> qbar[a]) & 1 for a in range(prog.n_atoms) if (negm >> a) & 1)

    gbits = guess  # the qbar atoms: constant self-loop rows
    atoms = 0
    news = 0
    for h, rs in by_head.items():  # v0: the fact rows
        for r in rs:
            if rules[r][1] == 0 and rules[r][2] == 0:
                if len(rs) == 1:
                    atoms |= 1 << h
                else:
                    news |= 1 << r
    products = 0
    while True:
        products += 1
        n_atoms, n_news = 0, 0
        for h, rs in by_head.items():
            if len(rs) == 1:
                if body_true(rs[0], atoms, gbits):
                    n_atoms |= 1 << h
            else:
                if any((news >> r) & 1 for r in rs):
                    n_atoms |= 1 << h
                for r in rs:
                    if body_true(r, atoms, gbits):
                        n_news |= 1 << r
        if n_atoms == atoms and n_news == news:
            return products
        atoms, news = n_atoms, n_news
