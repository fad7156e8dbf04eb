"""The dense-matrix method (lp_dense_least_model, lp_dense_stable_models):
the paper's third method of Section 4, Algorithms 1-3 with the program matrix
expanded to an n' x n' byte matrix.

It must give exactly the oracle's models and product counts: least models
against O1/O2, stable models (accepted guesses, models in guess order,
products) against O3, and the sparse engine's results at the stable-model
benchmark size (10,000 atoms, 16 negated atoms, 65,536 guesses), where the
product runs on the int8 matrix cores over 214 x 512 tiles."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2009_10247_amd import gen, lp
from tests import _golden

pytestmark = pytest.mark.gpu


def _check_least(prog):
    want, want_prods, _, _ = oracle.sd_fixpoint(prog)
    with lp.Matrix(prog) as m:
        got, prods, ms = m.dense_least_model()
    assert np.array_equal(got, want)
    assert prods == want_prods
    assert ms > 0
    return got, prods


def _check_stable(prog, max_models=4096):
    ref = oracle.stable(prog, want_interp=True)
    with lp.Matrix(prog) as m:
        res = m.dense_stable_models(max_models=max_models)
    acc = np.nonzero(ref["accept"])[0]
    assert np.array_equal(lp.accepted_indices(res["accepted"]), acc)
    assert res["n_models"] == acc.shape[0]
    assert res["products"] == ref["products"]
    for i, j in enumerate(acc[: res["models"].shape[0]]):
        w, b = divmod(int(j), 64)
        col = ((ref["interp"][:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)
        assert np.array_equal(res["models"][i], col), j
    return res


# ---------------------------------------------------------------- Algorithm 1

def test_example1_dense():
    d = _golden.load("example1.txt")
    with lp.Matrix(_golden.program(d)) as m:
        got, prods, _ = m.dense_least_model()
    assert [a for a, x in zip(d["atoms"], got) if x] == d["least_model"]
    assert prods == d["products"][0]


def test_tiny_programs_dense_match_brute_force():
    for seed in range(100):
        p = gen.tiny_random(seed, max_atoms=16, max_rules=40, max_body=4)
        with lp.Matrix(p) as m:
            got, prods, _ = m.dense_least_model()
        assert brute.from_vector(got) == brute.least_model(p), seed
        assert prods == oracle.sd_fixpoint(p)[1], seed


@pytest.mark.parametrize("n", [1, 63, 1000, 1023, 1025, 3000])
def test_dense_least_ragged_sizes(n):
    # n' crosses multiples of the 1024-byte padding and of the 32 rows a
    # workgroup takes
    _check_least(gen.definite_uniform(n, n, 3 * n, 0.05, 4))


def test_dense_least_1k_atoms_2k_rules():
    _check_least(gen.definite_uniform(0, 1000, 2000, 0.05, 4))


def test_dense_long_chain_products():
    # a 300-long chain: atom i turns true in product i, one more product
    # confirms the fixpoint; each product is one sweep of the dense matrix
    rules = [(0, [])] + [(i, [i - 1]) for i in range(1, 300)]
    got, prods = _check_least(gen.from_rules(300, rules))
    assert prods == 300 and got.all()


def test_dense_least_paper_shaped():
    # the definite-program table's sixth row (2,000 atoms, 40,000 rules), the
    # size the dense benchmark line uses
    _check_least(gen.paper_definite(0, 2000, 40000))


def test_dense_transitive_closure():
    edges = gen.random_graph_edges(3, 40, 120)
    _check_least(gen.transitive_closure(40, edges, grounding="all"))


def test_dense_empty_and_fact_only():
    empty = gen.Program(0, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32))
    with lp.Matrix(empty) as m:
        got, prods, _ = m.dense_least_model()
    assert got.shape == (0,) and prods == 1
    _check_least(gen.from_rules(5, []))
    _check_least(gen.from_rules(5, [(1, []), (3, []), (1, [])]))


def test_dense_least_rejects_negation():
    p = gen.from_rules(2, [(0, [gen.neg(1)])])
    with lp.Matrix(p) as m:
        with pytest.raises(lp.LPError) as e:
            m.dense_least_model()
        assert e.value.code == lp.LP_E_NEGATION


def test_dense_too_large_is_nomem():
    # 3,000,000 atoms: a dense matrix of 9 x 10^12 bytes cannot fit; the
    # check fails before any allocation and the library stays usable
    p = gen.from_rules(3_000_000, [(0, [])])
    with lp.Matrix(p) as m:
        with pytest.raises(lp.LPError) as e:
            m.dense_least_model()
        assert e.value.code == lp.LP_E_NOMEM
    _check_least(gen.definite_uniform(1, 200, 400, 0.05, 4))


def test_dense_host_only_rejected():
    p = gen.definite_uniform(2, 100, 200)
    with lp.Matrix(p, flags=lp.LP_BUILD_HOST_ONLY) as m:
        with pytest.raises(lp.LPError) as e:
            m.dense_least_model()
        assert e.value.code == lp.LP_E_HOST_ONLY


# ---------------------------------------------------------------- Algorithms 2 and 3

def test_example2_dense():
    d = _golden.load("example2.txt")
    p = _golden.program(d)
    res = _check_stable(p)
    assert [[a for a, x in zip(d["atoms"], mdl) if x] for mdl in res["models"]] == [["t"]]
    assert list(lp.accepted_indices(res["accepted"])) == d["accepted_guesses"]


def test_tiny_normal_programs_dense_match_brute_force():
    for seed in range(80):
        p = gen.tiny_random(40_000 + seed, max_atoms=9, max_rules=16, max_body=3, p_neg=0.35)
        res = _check_stable(p)
        got = sorted(brute.from_vector(m) for m in res["models"])
        assert got == brute.stable_models(p), seed


@pytest.mark.parametrize("k", [1, 3, 6, 7, 8, 9, 12])
def test_dense_stable_each_guess_width(k):
    # 2^k columns: below one 128-column tile, exactly one, and several
    _check_stable(gen.normal_uniform(k, 600, 1200, 5, k_neg=k, p_neg=0.2))


@pytest.mark.parametrize("n", [1, 4, 6])
def test_dense_even_loops(n):
    assert _check_stable(gen.even_loops(n))["n_models"] == 2 ** n


def test_dense_odd_loop_and_definite():
    with lp.Matrix(gen.odd_loop()) as m:
        assert m.dense_stable_models()["n_models"] == 0
    p = gen.definite_uniform(3, 400, 800)
    with lp.Matrix(p) as m:
        res = m.dense_stable_models()
    assert res["n_models"] == 1 and np.array_equal(res["models"][0], oracle.least_model(p))


def test_dense_stable_paper_shaped():
    # the normal-program table's sixth row: 2,000 atoms, 40,000 rules, 8
    # negated body literals
    _check_stable(gen.paper_normal(0, 2000, 40000, 8))


def test_dense_truncation():
    with lp.Matrix(gen.even_loops(5)) as m:
        res = m.dense_stable_models(max_models=7)
        full = m.stable_models(max_models=7)
    assert res["truncated"] and res["n_models"] == 32 and res["models"].shape[0] == 7
    assert np.array_equal(res["models"], full["models"])


def test_dense_equals_sparse_at_16_negated_atoms():
    # 10,000 atoms, 20,000 rules, 16 negated atoms: 65,536 guess columns
    p = gen.normal_uniform(0)
    with lp.Matrix(p) as m:
        dense = m.dense_stable_models(max_models=64)
        sparse = m.stable_models(max_models=64)
    assert np.array_equal(dense["accepted"], sparse["accepted"])
    assert dense["n_models"] == sparse["n_models"]
    assert dense["products"] == sparse["products"]
    assert np.array_equal(dense["models"], sparse["models"])
    for mdl in dense["models"]:
        assert oracle.gl_check(p, mdl)
