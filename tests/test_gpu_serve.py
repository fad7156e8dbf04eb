"""The native request loop (lp_server_*) through the C-ABI: every result in a
mixed stream (batched, concurrent, with evictions) equals the same request
solved alone, and the alone results equal the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp, serve

pytestmark = pytest.mark.gpu


def _pool():
    # least and stable queries (K up to 6), atoms 200..20,000
    return gen.serving_pool(3, 24, lo=200, hi=20_000, max_k=6)


def _check_alone_vs_oracle(pool, pids, ref):
    for p, pid in zip(pool, pids):
        model, acc, prods, n_models = ref[pid]
        if (p.body_lit < 0).any():
            want = oracle.stable(p, want_interp=True)
            acc_o = np.nonzero(want["accept"])[0]
            assert np.array_equal(lp.accepted_indices(acc), acc_o), pid
            assert n_models == acc_o.shape[0] and prods == want["products"], pid
            if acc_o.shape[0]:
                w, b = divmod(int(acc_o[0]), 64)
                first = ((want["interp"][:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)
                assert np.array_equal(model, first), pid
            else:
                assert not model.any()
        else:
            lm, wp, _, _ = oracle.sd_fixpoint(p)
            assert np.array_equal(model, lm) and prods == wp, pid


def test_stream_results_equal_alone_and_oracle():
    pool = _pool()
    with lp.Server(n_slots=6) as srv:
        pids = [srv.add_program(p) for p in pool]
        ref = serve.solve_alone(srv, pids)
        _check_alone_vs_oracle(pool, pids, ref)
        w = serve.zipf_weights(len(pids))
        # a burst (arrivals far faster than service): requests pile up, batch and overlap
        row = serve.run_stream(srv, pids, w, rate=1e6, n_requests=400, seed=1, ref=ref)
        assert row["mismatches"] == 0
        assert row["batched"] > 0
        row2 = serve.run_stream(srv, pids, w, rate=200.0, n_requests=100, seed=2, ref=ref)
        assert row2["mismatches"] == 0
        st = srv.stats()
        assert st["completed"] == len(pids) + 500 and st["pending"] == 0
        assert st["n_resident"] == len(pids) and st["uploads"] == len(pids)


def test_stable_requests_batch_under_load():
    # small stable programs (at most 12 negated atoms, small interpretation
    # matrices) join stable-model batches when requests pile up; the larger
    # ones run alone; every result equals the request solved alone
    pool = [gen.normal_uniform(90 + s, 300 + 100 * s, 600 + 200 * s, 4, 1 + s % 10, 0.1, 2, 0.02) for s in range(12)]
    pool += [gen.normal_uniform(110, 5_000, 10_000, 5, 12, 0.1, 2, 0.02), gen.definite_uniform(111, 2000, 4000, 0.02, 4)]
    with lp.Server(n_slots=1) as srv:
        pids = [srv.add_program(p) for p in pool]
        ref = serve.solve_alone(srv, pids)
        _check_alone_vs_oracle(pool, pids, ref)
        row = serve.run_stream(srv, pids, np.full(len(pids), 1.0 / len(pids)), rate=1e6, n_requests=200, seed=11,
                               ref=ref)
        assert row["mismatches"] == 0
        assert row["batched_stable"] > 0


def test_small_budget_evicts_and_results_still_equal():
    pool = _pool()
    with lp.Server(n_slots=4) as big:
        pids = [big.add_program(p) for p in pool]
        ref = serve.solve_alone(big, pids)
    # room for a few matrices at a time (each request is also charged about
    # 2 MiB of slack for its solve buffers and the allocator's rounding)
    with lp.Matrix(max(pool, key=lambda p: p.n_literals)) as m:
        largest = m.info["device_bytes"]
    budget = 4 * largest + (8 << 20)
    with lp.Server(n_slots=4, hbm_budget=budget) as srv:
        pids2 = [srv.add_program(p) for p in pool]
        assert pids2 == pids
        w = np.full(len(pids), 1.0 / len(pids))
        row = serve.run_stream(srv, pids, w, rate=1e6, n_requests=300, seed=5, ref=ref)
        assert row["mismatches"] == 0
        st = srv.stats()
        assert st["evictions"] > 0 and st["peak_used_bytes"] <= budget


def test_no_batching_gives_same_results():
    pool = _pool()
    with lp.Server(n_slots=3, batch_max=1) as srv:
        pids = [srv.add_program(p) for p in pool]
        ref = serve.solve_alone(srv, pids)
        row = serve.run_stream(srv, pids, serve.zipf_weights(len(pids)), rate=1e6, n_requests=150, seed=7,
                               ref=ref)
        assert row["mismatches"] == 0 and row["batched"] == 0


def test_server_argument_errors():
    with lp.Server(n_slots=1) as srv:
        with pytest.raises(lp.LPError) as e:
            srv.submit(0)
        assert e.value.code == lp.LP_E_INVAL
        with pytest.raises(lp.LPError) as e:
            srv.add_program(gen.from_rules(30, [(0, [gen.neg(i) for i in range(1, 26)])]))
        assert e.value.code == lp.LP_E_TOO_MANY_GUESSES
        with pytest.raises(lp.LPError) as e:
            srv.add_program(gen.from_rules(2, [(5, [])]))
        assert e.value.code == lp.LP_E_INVAL
        assert srv.wait_any(10) is None


def test_matrix_evict_and_upload_round_trip():
    p = gen.definite_uniform(8, 3000, 6000, 0.02, 5)
    lm, wp, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        before = m.info["device_bytes"]
        m.evict()
        assert m.info["device_bytes"] == 0
        with pytest.raises(lp.LPError) as e:
            m.least_model()
        assert e.value.code == lp.LP_E_HOST_ONLY
        m.upload()
        assert m.info["device_bytes"] == before
        g, pr = m.least_model()
        assert np.array_equal(g, lm) and pr == wp
    st = lp.memory_stats()
    assert st["in_use"] >= 0 and st["cached"] >= 0


def test_resident_bytes_count_the_transposed_matrix():
    # stable programs of >= 2^19 row-words solve by dirty rows, whose
    # transposed matrix is uploaded with the matrix: the server's accounted
    # bytes must equal what the resident matrices really hold
    pool = [gen.normal_uniform(80 + s, 10_000, 20_000, 5, k_neg=12, p_neg=0.1) for s in range(2)]
    pool += [gen.definite_uniform(82, 50_000, 100_000, 0.02, 5), gen.normal_uniform(83, 300, 600, 4, k_neg=5)]
    with lp.Server(n_slots=2) as srv:
        pids = [srv.add_program(p) for p in pool]
        ref = serve.solve_alone(srv, pids)
        row = serve.run_stream(srv, pids, np.full(len(pids), 1.0 / len(pids)), rate=1e6, n_requests=40,
                               seed=3, ref=ref)
        assert row["mismatches"] == 0
        st = srv.stats()
    assert st["evictions"] == 0 and st["n_resident"] == len(pool)
    want = 0
    for p in pool:
        with lp.Matrix(p) as m:
            if m.info["n_neg"]:
                upload_bytes = m.info["device_bytes"]
                m.stable_models(max_models=1)
                # the stable-solve plan (two interpretation matrices and lists) is kept with the matrix
                assert m._info()["device_bytes"] >= upload_bytes
            else:
                m.least_model()
            want += m._info()["device_bytes"]
            if p.n_atoms == 10_000:  # dirty rows: the transposed matrix is part of the upload
                with lp.Matrix(p, flags=lp.LP_STABLE_FULL_SWEEP) as full:
                    assert full.info["device_bytes"] + 4 * m.info["nnz"] < upload_bytes
    assert st["used_bytes"] == want
