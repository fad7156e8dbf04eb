"""Seeded generators: the structural properties their docstrings state."""
import numpy as np
import pytest

from paper_2009_10247_amd import gen, serve


@pytest.mark.parametrize("seed", range(4))
def test_vectorized_negations_respect_constraints(seed):
    p = gen.normal_uniform(seed, 3000, 9000, 6, 12, 0.1, 2, 0.02, vectorized=True)
    lit = p.body_lit.astype(np.int64)
    negs = np.unique(-lit[lit < 0] - 1)
    assert negs.shape[0] == 12
    for r in range(p.n_rules):
        a, b = int(p.body_ptr[r]), int(p.body_ptr[r + 1])
        body = lit[a:b]
        q = -body[body < 0] - 1
        assert q.shape[0] <= 2
        assert np.unique(q).shape[0] == q.shape[0]          # distinct negated atoms
        assert not np.isin(q, body[body >= 0]).any()        # not also positive
        assert not (q == p.head[r]).any()                   # not the head


def test_vectorized_negation_rate():
    p = gen.normal_uniform(1, 20_000, 60_000, 6, 12, 0.1, 2, 0.0, vectorized=True)
    lit = p.body_lit
    per_rule = np.add.reduceat((lit < 0).astype(np.int64), p.body_ptr[:-1])
    frac = float((per_rule > 0).mean())
    assert 0.08 < frac < 0.12


def test_serving_pool_kinds_and_sizes():
    pool = gen.serving_pool(0, 40, lo=100, hi=5000)
    ks = [int(np.unique(-p.body_lit[p.body_lit < 0].astype(np.int64) - 1).shape[0]) for p in pool]
    assert all(0 <= k <= 12 for k in ks) and any(k == 0 for k in ks) and any(k > 0 for k in ks)
    for p in pool:
        assert 100 <= p.n_atoms <= 5000 and p.n_rules == 3 * p.n_atoms


def test_batch_programs_sizes_and_seeds():
    a = gen.batch_programs(0, 16)
    b = gen.batch_programs(0, 16)
    assert all(np.array_equal(x.body_lit, y.body_lit) for x, y in zip(a, b))
    for p in a:
        assert 1000 <= p.n_atoms <= 100_000 and p.n_rules == 2 * p.n_atoms
        L = np.diff(p.body_ptr)
        assert L.max() <= 6 and abs(float((L == 0).mean()) - 0.02) < 0.02


def test_zipf_weights():
    w = serve.zipf_weights(256)
    assert abs(w.sum() - 1.0) < 1e-12 and (np.diff(w) < 0).all()
    assert abs(w[0] / w[1] - 2.0) < 1e-12
