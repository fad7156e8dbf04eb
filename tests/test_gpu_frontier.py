"""The frontier driver (semi-naive push through the transposed matrix):
same least models and product counts as the oracle and the full-sweep
drivers. The parametrized parity tests of test_gpu_parity.py also run it
(schedule "frontier")."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu

FRONTIER = lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER)
BATCHED = lp.make_schedule(driver=lp.LP_DRIVER_BATCHED)


def test_full_size_chain_zipf():
    # the benchmarked workload: 1,000,000 atoms, 5,000,000 rules, 2,000-long chain
    p = gen.chain_zipf(0)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        got, prods = m.least_model(sched=FRONTIER)
        assert np.array_equal(got, want) and prods == want_prods == 2000
        again, prods2 = m.least_model(sched=FRONTIER)  # the transpose is reused
        assert np.array_equal(again, want) and prods2 == 2000


@pytest.mark.parametrize("seed", range(6))
def test_same_as_full_sweep(seed):
    for p in gen.batch_programs(100 + seed, count=8, lo=50, hi=20_000):
        with lp.Matrix(p) as m:
            a, pa = m.least_model(sched=FRONTIER)
            b, pb = m.least_model(sched=BATCHED)
        assert np.array_equal(a, b) and pa == pb


def test_hub_atoms_with_long_occurrence_lists():
    # atom 0 is named by 50,000 bodies and atom 1 by 70,000 (lists longer than a
    # wave's pass many times over), mixed with short lists in the same chunk
    rng = np.random.default_rng(3)
    n = 120_000
    rules = [(0, []), (1, [0])]
    rules += [(int(h), [0, int(b)]) for h, b in zip(rng.integers(2, n, 50_000), rng.integers(2, 200, 50_000))]
    rules += [(int(h), [1]) for h in rng.integers(200, n, 70_000)]
    rules += [(int(h), []) for h in rng.integers(2, 200, 30)]
    p = gen.from_rules(n, rules)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        got, prods = m.least_model(sched=FRONTIER)
    assert np.array_equal(got, want) and prods == want_prods


def test_after_evict_and_upload():
    p = gen.chain_zipf(5, n_atoms=20_000, n_rules=100_000, chain_len=60)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        assert np.array_equal(m.least_model(sched=FRONTIER)[0], want)
        m.evict()
        m.upload()
        got, prods = m.least_model(sched=FRONTIER)
    assert np.array_equal(got, want) and prods == want_prods == 60


def test_unknown_driver_is_an_error():
    with lp.Matrix(gen.definite_uniform(0, 100, 200)) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model(sched=lp.make_schedule(driver=9))
        assert e.value.code == lp.LP_E_INVAL


@pytest.mark.parametrize("chain,bursts", [
    (400, ()), (400, (15,)), (400, (16,)), (400, (17, 150)), (400, (15, 16, 100, 101, 300)), (400, (271,)),
    (700, (100, 200, 600)), (127, ()), (128, ()), (270, ()), (271, ()), (272, ()), (527, ()), (528, ())])
def test_long_chain_with_bursts(chain, bursts):
    # a derivation chain (frontiers of a row or two, which one workgroup
    # takes in a loop over many levels) with bursts of 5,000 rows fired by
    # chain atom k for each k in `bursts` (a burst is F_{k+1}): a burst is
    # larger than the loop takes, so the full grid takes over at that level,
    # for 16 levels, and hands back after them. The first 16 levels run on
    # the full grid and the loop takes levels 16-271 in its first launch.
    # Bursts at 15/16/17 put the large frontier just before, at and just
    # after the loop's start, 271 at the end of its first launch; chains of
    # 270-272 and 527-528 atoms put the fixpoint's empty frontier around the
    # ends of loop launches.
    burst = 5000
    n = chain + burst * len(bursts) + 1
    rules = [(0, [])] + [(i, [i - 1]) for i in range(1, chain)]
    base = chain
    for k in bursts:
        rules += [(base + j, [k]) for j in range(burst)]
        base += burst
    rules.append((n - 1, [chain - 1, base - 1 if bursts else 0]))
    p = gen.from_rules(n, rules)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        got, prods = m.least_model(sched=FRONTIER)
        b, pb = m.least_model(sched=BATCHED)
    assert np.array_equal(got, want) and prods == want_prods
    assert np.array_equal(b, want) and pb == want_prods
    assert got.all()
