"""The schedule cache on the GPU: lp_tune_schedule stores its schedule under
the matrix's size bucket; default solves of matrices in that bucket use it
and still equal the oracle; the cache survives a save / clear / load; the
server with tuning on tunes a new bucket once."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp, serve

pytestmark = pytest.mark.gpu


def _prog(seed):
    # past the one-workgroup loop (more than 131,072 entries + rows)
    return gen.definite_uniform(seed, 40_000, 80_000, 0.02, 4)


def test_tuned_schedule_serves_its_bucket(tmp_path):
    lp.schedule_cache_clear()
    a, b = _prog(1), _prog(2)
    with lp.Matrix(a) as ma, lp.Matrix(b) as mb:
        assert lp.schedule_cache_lookup(ma)[0] == 0
        sched, _, _ = ma.tune(reps=2)
        found, s = lp.schedule_cache_lookup(mb)  # same sizes: same bucket
        assert found == 1
        assert lp.schedule_dict(s) == lp.schedule_dict(sched)
        for m, p in ((ma, a), (mb, b)):
            want, wp, _, _ = oracle.sd_fixpoint(p)
            got, pr = m.least_model()
            assert np.array_equal(got, want) and pr == wp
        path = tmp_path / "cache.txt"
        lp.schedule_cache_save(str(path))
        lp.schedule_cache_clear()
        assert lp.schedule_cache_lookup(ma)[0] == 0
        lp.schedule_cache_load(str(path))
        assert lp.schedule_cache_lookup(ma)[0] == 1
    with lp.Matrix(gen.definite_uniform(3, 1000, 2000, 0.05, 4)) as small:
        assert lp.schedule_cache_lookup(small)[0] == 2
    with lp.Matrix(gen.normal_uniform(4, 300, 600, 4, 3)) as normal:
        assert lp.schedule_cache_lookup(normal)[0] == 0
    lp.schedule_cache_clear()


def test_server_tunes_a_new_bucket_once():
    lp.schedule_cache_clear()
    pool = [_prog(10), _prog(11), gen.definite_uniform(12, 1000, 2000, 0.05, 4)]
    with lp.Server(n_slots=1, tune=True) as srv:
        pids = [srv.add_program(p) for p in pool]
        ref = serve.solve_alone(srv, pids)
        for p, pid in zip(pool, pids):
            lm, wp, _, _ = oracle.sd_fixpoint(p)
            assert np.array_equal(ref[pid][0], lm) and ref[pid][2] == wp
        assert srv.stats()["tunes"] == 1
        row = serve.run_stream(srv, pids, np.full(len(pids), 1 / 3), rate=1e6, n_requests=30, seed=1, ref=ref)
        assert row["mismatches"] == 0 and srv.stats()["tunes"] == 1
    lp.schedule_cache_clear()
