"""Stable models of several programs in shared launches
(lp_stable_models_batch): every program's accepted guesses, model count,
first model and product count equal the oracle's (O3) and lp_stable_models'
with one model; programs outside the batched path (no negation, more than 12
negated atoms left after pruning) are solved alone in the same call."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu


def _want(p):
    r = oracle.stable(p, want_interp=True)
    acc = np.nonzero(r["accept"])[0]
    first = None
    if acc.shape[0]:
        w, b = divmod(int(acc[0]), 64)
        first = ((r["interp"][:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)
    return acc, first, r["products"]


def _check(progs, flags=None):
    flags = flags or [0] * len(progs)
    mats = [lp.Matrix(p, flags=f) for p, f in zip(progs, flags)]
    try:
        got = lp.stable_models_batch(mats)
        for i, (p, m, g) in enumerate(zip(progs, mats, got)):
            alone = m.stable_models(max_models=1)
            assert np.array_equal(g["accepted"], alone["accepted"]), i
            assert g["n_models"] == alone["n_models"] and g["products"] == alone["products"], i
            if alone["n_models"]:
                assert np.array_equal(g["model"], alone["models"][0]), i
            else:
                assert g["model"] is None
            if flags[i] == 0 and m.info["n_neg"] > 0:
                acc, first, prods = _want(p)
                assert np.array_equal(lp.accepted_indices(g["accepted"]), acc), i
                assert g["products"] == prods, i
                if first is not None:
                    assert np.array_equal(g["model"], first), i
        return got
    finally:
        for m in mats:
            m.close()


def test_small_programs_of_every_width():
    # K = 1..12: one to 64 words per row, with facts and without
    progs = [gen.normal_uniform(500 + k, 300 + 40 * k, 600 + 80 * k, 4, k, 0.1, 2, 0.02 * (k % 2)) for k in range(1, 13)]
    _check(progs)


def test_mixed_with_programs_solved_alone():
    progs = [gen.normal_uniform(600, 400, 800, 4, 5, 0.1, 2, 0.02),
             gen.definite_uniform(601, 500, 1000, 0.05, 4),       # no negation: alone
             gen.normal_uniform(602, 300, 600, 4, 14, 0.1, 2),     # 14 negated atoms: alone
             gen.even_loops(6), gen.odd_loop(),
             gen.normal_uniform(603, 2000, 4000, 5, 9, 0.1, 2, 0.02)]
    got = _check(progs)
    assert got[3]["n_models"] == 64 and got[4]["n_models"] == 0


def test_pruned_guesses_and_repeated_matrices():
    p = gen.normal_uniform(700, 500, 1000, 4, 10, 0.2, 2, 0.05)
    progs = [p, p, gen.normal_uniform(701, 800, 1600, 4, 7, 0.1, 2, 0.05)]
    _check(progs, flags=[lp.LP_PRUNE_FACT_GUESSES, 0, lp.LP_PRUNE_FACT_GUESSES])


def test_many_programs_and_long_fixpoints():
    # forty programs; a negation-gated chain of 300 makes one fixpoint far
    # longer than the others (products past the others' fixpoints skip them)
    progs = [gen.normal_uniform(800 + i, 200 + 25 * i, 400 + 50 * i, 4, 1 + i % 12, 0.1, 2, 0.02) for i in range(40)]
    L = 300
    chain = [(0, [gen.neg(L + 1)])] + [(i, [i - 1]) for i in range(1, L)]
    progs.insert(17, gen.from_rules(L + 2, chain))
    got = _check(progs)
    assert got[17]["products"] == L + 1


def test_empty_and_argument_errors():
    assert lp.stable_models_batch([]) == []
    p = gen.normal_uniform(900, 300, 600, 4, 3)
    with lp.Matrix(p) as m:
        L = lp.load()
        hs = (ctypes.c_void_p * 1)(m.handle.value)
        acc = np.zeros(1, dtype=np.uint64)
        nm = np.zeros(1, dtype=np.int64)
        aps = (ctypes.c_void_p * 1)(acc.ctypes.data)
        assert L.lp_stable_models_batch(hs, 1, None, nm.ctypes.data, None, None, None) == lp.LP_E_INVAL
        assert L.lp_stable_models_batch(hs, 1, aps, None, None, None, None) == lp.LP_E_INVAL
        assert L.lp_stable_models_batch(hs, -1, aps, nm.ctypes.data, None, None, None) == lp.LP_E_INVAL
        nulls = (ctypes.c_void_p * 1)(None)
        assert L.lp_stable_models_batch(hs, 1, nulls, nm.ctypes.data, None, None, None) == lp.LP_E_INVAL
        # models and products may be NULL
        assert L.lp_stable_models_batch(hs, 1, aps, nm.ctypes.data, None, None, None) == lp.LP_OK
        assert nm[0] == m.stable_models(max_models=1)["n_models"]
