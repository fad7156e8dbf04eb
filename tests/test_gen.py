"""Seeded generators: the structural properties their docstrings state."""
import numpy as np
import pytest

import oracle
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


def test_paper_definite_shape():
    p = gen.paper_definite(3, 2000, 36000)
    L = np.diff(p.body_ptr)
    n_facts = int((L == 0).sum())
    assert n_facts == (2000 - 1) // 3 and n_facts < 2000 / 3
    assert len(set(p.head[L == 0].tolist())) == n_facts  # distinct fact atoms
    body = L[L > 0]
    for length, q in enumerate(gen.PAPER_BODY_PROPORTIONS, 1):
        assert abs((body == length).mean() - q) < 0.002, length
    for r in range(0, p.n_rules, 97):  # bodies: distinct atoms, never the head
        lits = p.body_lit[p.body_ptr[r]:p.body_ptr[r + 1]]
        assert len(set(lits.tolist())) == lits.shape[0] and p.head[r] not in lits and (lits >= 0).all()


def test_paper_normal_negations():
    p = gen.paper_normal(4, 1000, 5000, 7)
    assert int((p.body_lit < 0).sum()) == 7
    base = gen.paper_definite(4, 1000, 5000)
    assert np.array_equal(np.where(p.body_lit < 0, -p.body_lit - 1, p.body_lit), base.body_lit)


def test_transitive_closure_all_grounding_is_warshall():
    # the all-triples grounding of path/edge: its least model's path atoms are
    # the transitive closure (Warshall's algorithm on the adjacency matrix)
    V = 9
    edges = gen.random_graph_edges(2, V, 14)
    p = gen.transitive_closure(V, edges, grounding="all")
    assert p.n_atoms == 2 * V * V and p.n_rules == V ** 3 + V * V + len(edges)
    model = oracle.least_model(p)
    reach = np.zeros((V, V), dtype=bool)
    for x, y in edges:
        reach[x, y] = True
    for z in range(V):
        reach |= reach[:, [z]] & reach[[z], :]
    assert np.array_equal(model[V * V:].reshape(V, V).astype(bool), reach)
