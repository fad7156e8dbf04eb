"""Stable models by dirty rows through the matrix's solve plan (buffers kept
between solves and restored to the initial matrix after each, a captured
graph for the first products): every replay equals the oracle, also when
solves of other matrices, full sweeps and concurrent solves of the same
matrix come in between, and when the fixpoint needs more products than the
graph holds."""
import threading

import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu


def _ref(p):
    return oracle.stable(p, want_interp=True)


def _same(res, ref):
    return (np.array_equal(lp.accepted_indices(res["accepted"]), np.nonzero(ref["accept"])[0])
            and np.array_equal(res["interp"], ref["interp"]) and res["products"] == ref["products"])


def test_replays_interleaved_with_other_work():
    pa = gen.normal_uniform(91, 3000, 6000, 4, k_neg=10, p_neg=0.15)
    pb = gen.normal_uniform(92, 2000, 4000, 5, k_neg=8, p_neg=0.15)
    ra, rb = _ref(pa), _ref(pb)
    with lp.Matrix(pa, flags=lp.LP_STABLE_DIRTY_ROWS) as ma, lp.Matrix(pb, flags=lp.LP_STABLE_DIRTY_ROWS) as mb, \
            lp.Matrix(pa, flags=lp.LP_STABLE_FULL_SWEEP) as mf:
        for it in range(5):
            assert _same(ma.stable_models(want_interp=True), ra), it
            assert _same(mb.stable_models(want_interp=True), rb), it
            assert _same(mf.stable_models(want_interp=True), ra), it
            g = gen.definite_uniform(it, 500, 1000)
            with lp.Matrix(g) as mg:
                want, wp, _, _ = oracle.sd_fixpoint(g)
                got, pr = mg.least_model()
                assert np.array_equal(got, want) and pr == wp
        # models in guess order, truncated
        res = ma.stable_models(max_models=1)
        assert res["n_models"] == int(ra["accept"].sum())


@pytest.mark.parametrize("L", [15, 16, 17, 40])
def test_more_products_than_the_graph_holds(L):
    # h_0 <- not x, h_i <- h_{i-1}, plus an even loop: L + 1 products
    x = L
    rules = [(0, [gen.neg(x)])] + [(i, [i - 1]) for i in range(1, L)]
    rules += [(L + 1, [gen.neg(L + 2)]), (L + 2, [gen.neg(L + 1)])]
    p = gen.from_rules(L + 3, rules)
    ref = _ref(p)
    assert ref["products"] == L + 1
    with lp.Matrix(p, flags=lp.LP_STABLE_DIRTY_ROWS) as m:
        for _ in range(3):
            assert _same(m.stable_models(want_interp=True), ref)


def test_concurrent_solves_of_one_matrix():
    import torch

    p = gen.normal_uniform(93, 4000, 8000, 4, k_neg=9, p_neg=0.15)
    ref = _ref(p)
    errors = []
    with lp.Matrix(p, flags=lp.LP_STABLE_DIRTY_ROWS) as m:
        streams = [torch.cuda.Stream() for _ in range(4)]

        def work(k):
            try:
                for _ in range(6):
                    if not _same(m.stable_models(want_interp=True, stream=streams[k]), ref):
                        errors.append(k)
            except BaseException as e:  # noqa: BLE001
                errors.append(repr(e))

        threads = [threading.Thread(target=work, args=(k,)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
    assert errors == []


def test_plan_survives_evict_and_upload():
    p = gen.normal_uniform(94, 2500, 5000, 4, k_neg=7, p_neg=0.2)
    ref = _ref(p)
    with lp.Matrix(p, flags=lp.LP_STABLE_DIRTY_ROWS) as m:
        assert _same(m.stable_models(want_interp=True), ref)
        grown = m._info()["device_bytes"]
        m.evict()
        m.upload()
        assert m._info()["device_bytes"] < grown  # the plan went with the device copy
        assert _same(m.stable_models(want_interp=True), ref)
        assert _same(m.stable_models(want_interp=True), ref)
