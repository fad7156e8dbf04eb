"""Stable models on caller-chosen guesses (lp_stable_models_guesses) and by
guess sampling with local search (lp_stable_models_search).

Per-guess results are exact against the oracle's per-guess least models
(O3): acceptance, the guess each fixpoint points to, and the models. The
search is sound (every model it returns passes the Gelfond-Lifschitz check
and, where the guesses can be enumerated, is among the oracle's models);
its completeness is not pinned."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu


def _column(interp, j):
    w, b = divmod(int(j), 64)
    return ((interp[:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)


@pytest.mark.parametrize("flags", [0, lp.LP_STABLE_DIRTY_ROWS])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_given_guesses_match_oracle(seed, flags):
    p = gen.normal_uniform(seed, 600, 1200, 5, k_neg=10, p_neg=0.2)
    ref = oracle.stable(p, want_interp=True)
    q = ref["neg_atoms"]
    K = q.shape[0]
    rng = np.random.default_rng(seed)
    acc_idx = np.nonzero(ref["accept"])[0]
    guesses = np.concatenate([rng.integers(0, 1 << K, size=300), acc_idx, acc_idx[:3]]).astype(np.uint64)
    with lp.Matrix(p, flags=flags) as m:
        res = m.stable_guesses(guesses, max_models=len(guesses))
    assert np.array_equal(res["accepted"], ref["accept"][guesses.astype(np.int64)].astype(bool))
    assert res["n_accepted"] == int(res["accepted"].sum())
    for j, g in enumerate(guesses.astype(np.int64)):
        col = _column(ref["interp"], g)
        want_next = sum(1 << t for t in range(K) if not col[q[t]])
        assert int(res["next"][j]) == want_next, j
    acc_guesses = guesses[res["accepted"]].astype(np.int64)
    for i, g in enumerate(acc_guesses):
        assert np.array_equal(res["models"][i], _column(ref["interp"], g))


def test_all_guesses_equal_enumeration():
    p = gen.normal_uniform(5, 800, 1600, 5, k_neg=9, p_neg=0.25)
    with lp.Matrix(p) as m:
        full = m.stable_models(want_interp=False)
        K = m.info["n_neg"]
        res = m.stable_guesses(np.arange(1 << K, dtype=np.uint64), want_next=False)
    assert np.array_equal(np.nonzero(res["accepted"])[0], lp.accepted_indices(full["accepted"]))
    assert res["products"] == full["products"]


def test_search_is_sound_where_enumerable():
    p = gen.even_loops(8)  # K = 16, 256 stable models
    ref = oracle.stable(p)
    with lp.Matrix(p) as m:
        res = m.stable_search(n_samples=2048, rounds=3, seed=7, max_found=4096)
        again = m.stable_search(n_samples=2048, rounds=3, seed=7, max_found=4096)
    assert res["n_found"] > 0 and not res["truncated"]
    assert np.all(ref["accept"][res["found"].astype(np.int64)] == 1)
    assert np.array_equal(res["found"], again["found"])  # same seed, same search
    for mdl in res["models"]:
        assert oracle.gl_check(p, mdl)


def test_search_beyond_enumeration():
    p = gen.even_loops(24)  # K = 48: 2^48 guesses, 2^24 stable models
    with lp.Matrix(p) as m:
        assert m.info["n_neg"] == 48
        res = m.stable_search(n_samples=4096, rounds=4, seed=1, max_found=256)
    assert res["n_found"] > 0
    for mdl in res["models"]:
        assert oracle.gl_check(p, mdl)
        assert np.all(mdl[0::2] != mdl[1::2])  # each loop picks exactly one of its two atoms


def test_search_finds_nothing_without_models():
    with lp.Matrix(gen.odd_loop()) as m:
        res = m.stable_search(n_samples=64, rounds=2, seed=3)
        g = m.stable_guesses(np.array([0, 1], dtype=np.uint64))
    assert res["n_found"] == 0 and g["n_accepted"] == 0


def test_guess_arguments_are_checked():
    with lp.Matrix(gen.even_loops(33)) as m:  # K = 66 > 64
        with pytest.raises(lp.LPError) as e:
            m.stable_guesses(np.zeros(4, dtype=np.uint64))
        assert e.value.code == lp.LP_E_TOO_MANY_GUESSES
    with lp.Matrix(gen.definite_uniform(0, 100, 200)) as m:  # K = 0
        with pytest.raises(lp.LPError) as e:
            m.stable_search()
        assert e.value.code == lp.LP_E_INVAL
    with lp.Matrix(gen.even_loops(3)) as m:
        with pytest.raises(lp.LPError) as e:
            m.stable_guesses(np.zeros(0, dtype=np.uint64))
        assert e.value.code == lp.LP_E_INVAL
