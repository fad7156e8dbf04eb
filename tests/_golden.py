"""Parser for the worked-example fixtures under tests/golden/."""
from __future__ import annotations

import os
from fractions import Fraction

from paper_2009_10247_amd import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    d: dict = dict(rules=[], matrix={}, guess_fixpoint={})
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(" ")
            toks = rest.split()
            if key == "rule":
                h, _, body = rest.partition("<-")
                d["rules"].append((h.strip(), body.split()))
            elif key == "matrix":
                d["matrix"][toks[0]] = [Fraction(t) for t in toks[1:]]
            elif key == "guess_fixpoint":
                d["guess_fixpoint"][int(toks[0])] = set(toks[1:])
            elif key == "stable_models":
                d["stable_models"] = [set(m.strip("{}").split(",")) - {""} for m in toks]
            elif key in ("coo_val", "csr_value"):
                d[key] = [float(t) for t in toks]
            elif key in ("coo_row", "coo_col", "csr_row_index", "csr_col_index",
                         "accepted_guesses", "products", "guess_products"):
                d[key] = [int(t) for t in toks]
            else:
                d[key] = toks
    return d


def program(d: dict) -> gen.Program:
    idx = {a: i for i, a in enumerate(d["atoms"])}
    rules = []
    for h, body in d["rules"]:
        lits = [gen.neg(idx[b[1:]]) if b.startswith("~") else idx[b] for b in body]
        rules.append((idx[h], lits))
    return gen.from_rules(len(d["atoms"]), rules, kind="golden")


def names_to_vector(names, atoms):
    return [1 if a in names else 0 for a in atoms]
