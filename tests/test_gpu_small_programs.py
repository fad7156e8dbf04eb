"""Least models of small programs under the default driver, which solves a
program of at most 64 words of rows (4,096 rows), 2,048 OR rows and no long
rows with every lane keeping its rows in registers (tp_tiny_kernel), and
slightly larger ones in one workgroup with the layout in LDS. Models and
product counts are compared with the CPU oracle (O2)."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu


def _check(p):
    want, wp, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        got, pr = m.least_model()
        info = m.info
    assert np.array_equal(got, want) and pr == wp
    return info


@pytest.mark.parametrize("seed", range(6))
def test_bodies_longer_than_the_registers_hold(seed):
    # bodies up to 8 entries: entries past the fourth come from LDS
    info = _check(gen.definite_uniform(200 + seed, 600, 1400, 0.05, 8))
    assert info["n_rows"] <= 4096


def _two_rules_per_head(seed, n_atoms, n_heads):
    # heads 0..n_heads-1 with two rules each (one OR row and two new rows per
    # head), the other atoms facts or single rules
    rng = np.random.default_rng(seed)
    rules = []
    for h in range(n_heads):
        for _ in range(2):
            body = rng.choice(n_atoms, size=int(rng.integers(1, 5)), replace=False)
            rules.append((h, [int(b) for b in body if b != h]))
    for a in range(n_heads, n_atoms):
        rules.append((a, []) if a % 7 == 0 else (a, [int(rng.integers(0, n_atoms))]))
    return gen.from_rules(n_atoms, rules)


@pytest.mark.parametrize("n_atoms,n_heads,words", [(1800, 1100, 63), (1850, 1100, 64), (1900, 1100, 65),
                                                    (1300, 1060, 54), (2100, 900, 61)])
def test_around_the_register_path_limits(n_atoms, n_heads, words):
    # row counts on both sides of 64 words (4,096 rows) and OR-row counts past
    # 1,024 (two per thread)
    for seed in range(3):
        info = _check(_two_rules_per_head(310 + seed, n_atoms, n_heads))
        assert (info["n_rows"] + 63) // 64 == words and info["n_or_rows"] == n_heads


@pytest.mark.parametrize("seed", range(4))
def test_uniform_programs_near_the_limit(seed):
    for n_atoms, n_rules in ((700, 3300), (800, 3600)):
        _check(gen.definite_uniform(300 + seed, n_atoms, n_rules, 0.03, 4))


def test_long_chain_of_products():
    # a 900-long derivation chain inside 1,000 atoms: 900 products in one launch
    L = 900
    rules = [(0, [])] + [(i, [i - 1]) for i in range(1, L)] + [(L + (i % 90), [i, (i * 7) % L]) for i in range(200)]
    info = _check(gen.from_rules(1000, rules))
    assert info["n_rows"] <= 4096


def test_or_rows_fire_once_and_stay():
    # heads with many rules (OR rows over their new atoms); facts among them
    rules = []
    for h in range(50):
        rules.append((h, []) if h % 10 == 0 else (h, [(h + 1) % 50]))
        for k in range(5):
            rules.append((h, [(h + k + 2) % 50, (h + 3 * k + 1) % 50]))
    _check(gen.from_rules(50, rules))


def test_no_facts_and_facts_only():
    _check(gen.definite_uniform(7, 500, 900, 0.0, 3))
    _check(gen.from_rules(40, [(i, []) for i in range(0, 40, 3)] + [(5, []), (5, [])]))


def test_self_loops_and_duplicates():
    rules = [(0, [0]), (1, []), (2, [1, 1, 1]), (3, [2, 3]), (3, [1]), (4, [3, 2, 1, 0]), (5, [4, 4])]
    _check(gen.from_rules(6, rules))
