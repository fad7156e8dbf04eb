"""Parity of the batched least-model kernel (many programs in one launch,
each workgroup running whole fixpoints from a device work queue) with the CPU
oracle, through the C-ABI. Models and product counts must match exactly, for
every shape, on graph replays and whatever the batch composition."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4), (4, 8), (4, 16), (8, 8), (8, 16)]


def _want(progs):
    return [oracle.sd_fixpoint(p)[:2] for p in progs]


def _assert_equal(got, want, tag=""):
    assert len(got) == len(want)
    for i, ((g, pr), (w, wp)) in enumerate(zip(got, want)):
        assert np.array_equal(g, w), (tag, i)
        assert pr == wp, (tag, i, pr, wp)


def _edge_programs():
    rng = np.random.default_rng(3)
    out = [
        gen.from_rules(0, []),                                   # no atoms
        gen.from_rules(1, []),                                   # one atom, no rule
        gen.from_rules(1, [(0, [])]),                            # one fact
        gen.from_rules(5, [(a, []) for a in range(5)]),          # facts only
        gen.from_rules(64, [(0, [])] + [(i, [i - 1]) for i in range(1, 64)]),   # chain over one word
        gen.from_rules(65, [(0, [])] + [(i, [i - 1]) for i in range(1, 65)]),   # ragged last word
        gen.from_rules(300, [(i, [i - 1]) for i in range(1, 300)]),             # no facts: empty model
    ]
    # long OR and AND rows (segment pass): one head with 10,000 rules, a
    # 9,000-atom body that fires and one that does not
    n = 20_000
    rules = [(a, []) for a in range(0, 12_000)]
    rules += [(19_000, [int(x)]) for x in rng.integers(12_000, 18_000, size=10_000)]
    rules += [(19_001, list(range(0, 9_000)))]
    rules += [(19_002, list(range(1, 9_000)) + [19_500])]
    rules += [(int(h), [int(b)]) for h, b in zip(rng.integers(12_000, 18_000, 3000), rng.integers(0, 12_000, 3000))]
    rules += [(19_003, [19_001, 19_000])]
    out.append(gen.from_rules(n, rules))
    # AND entries only past 5,000 fact rows (the waves' stretches of words
    # split by work leave the leading words to few waves), rows of 200-255
    # entries that span rounds and super-blocks, and a chain of 255-entry rows
    # (254 facts and the previous link) whose links fire one product apart
    rules = [(a, []) for a in range(5000)]
    rules += [(5000 + i, [int(x) for x in rng.choice(5000, size=int(rng.integers(200, 256)), replace=False)])
              for i in range(600)]
    rules += [(5600 + i, [int(x) for x in rng.choice(5000, size=254, replace=False)] + [5599 + i])
              for i in range(300)]
    rules += [(5900, [int(x) for x in rng.choice(5000, size=255, replace=False)] + [5950])]  # 256 entries, never fires
    out.append(gen.from_rules(6000, rules))
    return out


def test_batch_config_512_programs_vs_oracle():
    # 512 programs, atoms log-uniform in 1e3..1e5, 2x rules, bodies 1..6, 2% facts
    progs = gen.batch_programs(0, 512)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        with lp.Batch(mats) as b:
            info = b.info()
            assert info["count"] == 512 and info["n_resident"] == 512
            # the largest programs are split among teams of workgroups
            assert info["n_teams"] > 0 and info["team_members"] <= 256
            b.run()
            _assert_equal(b.results(), want, "default")
            b.tune(reps=1)
            b.run()
            _assert_equal(b.results(), want, "tuned")
            assert b.info()["team_fallbacks"] == 0
        _assert_equal(lp.least_model_batch(mats), want, "one call")
    finally:
        for m in mats:
            m.close()


@pytest.mark.parametrize("wpw,unroll", SHAPES)
@pytest.mark.parametrize("block", [256, 1024])
def test_batch_shapes(wpw, unroll, block):
    progs = gen.batch_programs(5, count=40, lo=50, hi=20_000) + _edge_programs()
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        sched = lp.make_schedule(wpw=wpw, unroll=unroll, block=block)
        _assert_equal(lp.least_model_batch(mats, sched=sched), want, (wpw, unroll, block))
    finally:
        for m in mats:
            m.close()


@pytest.mark.parametrize("seed", range(6))
def test_batch_random_plans(seed):
    # random programs (skewed sizes, chains, facts-only and OR-heavy ones) under
    # a random shape, block, grid and team setting; every model and product
    # count against the oracle
    rng = np.random.default_rng(100 + seed)
    progs = gen.batch_programs(200 + seed, count=int(rng.integers(8, 40)), lo=20, hi=int(rng.integers(500, 30_000)))
    L = int(rng.integers(2, 120))
    progs.append(gen.from_rules(L, [(0, [])] + [(i, [i - 1]) for i in range(1, L)]))
    n = int(rng.integers(200, 3000))
    progs.append(gen.from_rules(n, [(a, []) for a in range(n // 2)] +
                                [(int(h), [int(x)]) for h, x in zip(rng.integers(n // 2, n, 4 * n), rng.integers(0, n, 4 * n))]))
    order = rng.permutation(len(progs))
    progs = [progs[i] for i in order]
    want = _want(progs)
    wpw, unroll = SHAPES[int(rng.integers(len(SHAPES)))]
    block = int(rng.choice([256, 512, 1024]))
    team = int(rng.choice([0, 1, 2, 3]))
    grid = int(rng.choice([0, 0, 7, 64]))
    mats = [lp.Matrix(p) for p in progs]
    try:
        sched = lp.make_schedule(wpw=wpw, unroll=unroll, block=block, team=team, grid=grid)
        with lp.Batch(mats, sched=sched) as b:
            b.run()
            _assert_equal(b.results(), want, (seed, wpw, unroll, block, team, grid))
            b.run()
            _assert_equal(b.results(), want, (seed, "replay"))
    finally:
        for m in mats:
            m.close()


@pytest.mark.parametrize("grid", [1, 3])
def test_batch_few_workgroups_take_many_programs(grid):
    progs = gen.batch_programs(9, count=30, lo=20, hi=3000) + _edge_programs()
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        sched = lp.make_schedule(grid=grid)
        with lp.Batch(mats, sched=sched) as b:
            assert b.info()["grid"] == grid
            b.run()
            _assert_equal(b.results(), want, grid)
    finally:
        for m in mats:
            m.close()


def test_batch_graph_replays_with_work_between():
    progs = gen.batch_programs(21, count=64, lo=100, hi=30_000)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    other = gen.definite_uniform(99, 5000, 12_000, 0.02, 5)
    try:
        with lp.Batch(mats) as b, lp.Matrix(other) as mo:
            w_other = oracle.sd_fixpoint(other)[:2]
            for rep in range(3):
                b.run()
                _assert_equal(b.results(), want, rep)
                g, pr = mo.least_model()  # eager work between replays
                assert np.array_equal(g, w_other[0]) and pr == w_other[1]
            for rep in range(3):  # back-to-back replays, one read
                b.run()
            _assert_equal(b.results(), want, "back-to-back")
    finally:
        for m in mats:
            m.close()


def test_batch_results_independent_of_composition():
    progs = gen.batch_programs(33, count=48, lo=100, hi=50_000)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        alone = [lp.least_model_batch([m])[0] for m in mats]
        _assert_equal(alone, want, "alone")
        mixed = lp.least_model_batch(mats)
        _assert_equal(mixed, want, "mixed")
        perm = np.random.default_rng(1).permutation(len(mats))
        shuffled = lp.least_model_batch([mats[i] for i in perm])
        _assert_equal(shuffled, [want[i] for i in perm], "shuffled")
        single = [m.least_model() for m in mats]
        _assert_equal(single, want, "single-program driver")
    finally:
        for m in mats:
            m.close()


def test_batch_program_larger_than_lds_uses_single_driver():
    # ~820k matrix rows: two bit-packed buffers exceed a workgroup's LDS
    big = gen.definite_uniform(4, 300_000, 600_000, 0.02, 4)
    progs = [gen.definite_uniform(5, 2000, 4000, 0.02, 4), big, gen.definite_uniform(6, 3000, 6000, 0.02, 4)]
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        with lp.Batch(mats) as b:
            assert b.info()["n_resident"] == 2
            b.run()
            _assert_equal(b.results(), want)
    finally:
        for m in mats:
            m.close()


def test_batch_rejects_negation_and_accepts_empty():
    pos = gen.definite_uniform(1, 100, 200, 0.05, 3)
    negp = gen.from_rules(2, [(0, [gen.neg(1)])])
    with lp.Matrix(pos) as a, lp.Matrix(negp) as b:
        with pytest.raises(lp.LPError) as e:
            lp.least_model_batch([a, b])
        assert e.value.code == lp.LP_E_NEGATION
    assert lp.least_model_batch([]) == []
    with lp.Batch([]) as b:
        b.run()
        assert b.results() == []
        assert b.info()["n_resident"] == 0


def test_batch_unsupported_shape_rejected():
    p = gen.definite_uniform(1, 100, 200, 0.05, 3)
    with lp.Matrix(p) as m:
        with pytest.raises(lp.LPError) as e:
            lp.least_model_batch([m], sched=lp.make_schedule(wpw=2, unroll=8))
        assert e.value.code == lp.LP_E_INVAL
        with pytest.raises(lp.LPError) as e:
            lp.least_model_batch([m], sched=lp.make_schedule(block=128))
        assert e.value.code == lp.LP_E_INVAL


# ---------------------------------------------------------------- teams

@pytest.mark.parametrize("team", [2, 3, 8])
@pytest.mark.parametrize("wpw,unroll,block", [(4, 16, 1024), (4, 8, 256)])
def test_batch_forced_teams(team, wpw, unroll, block):
    # every program solved by a team of `team` workgroups: members take every
    # team-th super-block, OR row and segment, and meet after each product
    progs = gen.batch_programs(7, count=24, lo=50, hi=40_000) + _edge_programs()
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        sched = lp.make_schedule(wpw=wpw, unroll=unroll, block=block, team=team)
        with lp.Batch(mats, sched=sched) as b:
            info = b.info()
            assert info["n_teams"] == len(progs) and info["team_members"] == team * len(progs)
            for rep in range(2):
                b.run()
                _assert_equal(b.results(), want, (team, rep))
            assert b.info()["team_fallbacks"] == 0
    finally:
        for m in mats:
            m.close()


def test_batch_team_graph_replays_with_work_between():
    # team states are cleared by the last workgroup of each launch; replays of
    # the captured graph, with eager solves between them, give the same results
    progs = gen.batch_programs(23, count=16, lo=20_000, hi=60_000)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    other = gen.definite_uniform(98, 4000, 9000, 0.02, 5)
    try:
        with lp.Batch(mats, sched=lp.make_schedule(team=4)) as b, lp.Matrix(other) as mo:
            w_other = oracle.sd_fixpoint(other)[:2]
            for rep in range(3):
                b.run()
                _assert_equal(b.results(), want, rep)
                g, pr = mo.least_model()
                assert np.array_equal(g, w_other[0]) and pr == w_other[1]
            for rep in range(3):
                b.run()
            _assert_equal(b.results(), want, "back-to-back")
            assert b.info()["team_fallbacks"] == 0
    finally:
        for m in mats:
            m.close()


def test_batch_teams_off_and_small_grids():
    progs = gen.batch_programs(11, count=12, lo=1000, hi=80_000)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        with lp.Batch(mats, sched=lp.make_schedule(team=1)) as b:
            assert b.info()["n_teams"] == 0
            b.run()
            _assert_equal(b.results(), want, "off")
        # a grid of 4 workgroups allows teams of at most 2
        with lp.Batch(mats, sched=lp.make_schedule(grid=4, team=8)) as b:
            info = b.info()
            assert info["grid"] == 4 and info["team_members"] == 2 * len(progs)
            b.run()
            _assert_equal(b.results(), want, "grid 4")
        # one large program alone: a team of 8
        with lp.Batch(mats[:1]) as b:
            assert b.info()["team_members"] in (0, 8)
            b.run()
            _assert_equal(b.results(), want[:1], "alone")
    finally:
        for m in mats:
            m.close()


def test_batch_team_that_gives_up_is_solved_alone():
    # a team barrier bounded at one poll gives up whenever a member is not
    # already there; lp_batch_results then solves those programs alone, so the
    # results stay exact (the fallback path, forced from the host)
    progs = gen.batch_programs(13, count=20, lo=2000, hi=40_000)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        with lp.Batch(mats, sched=lp.make_schedule(team=4, team_polls=1)) as b:
            for rep in range(2):
                b.run()
                _assert_equal(b.results(), want, rep)
            assert b.info()["team_fallbacks"] > 0
        # and with the default bound nothing falls back
        with lp.Batch(mats, sched=lp.make_schedule(team=4)) as b:
            b.run()
            _assert_equal(b.results(), want, "default bound")
            assert b.info()["team_fallbacks"] == 0
    finally:
        for m in mats:
            m.close()


@pytest.mark.parametrize("team", [0, 3])
def test_batch_tune_lays_out_again_by_products(team):
    # lp_batch_tune's first call runs the batch and orders the queue and the
    # teams by product counts; the plan holds a program solved by the
    # single-program drivers too; a second tune keeps that layout
    big = gen.definite_uniform(4, 300_000, 600_000, 0.02, 4)
    progs = [gen.definite_uniform(40 + i, 1000 * (i + 1), 2000 * (i + 1), 0.02, 6) for i in range(20)]
    progs.insert(7, big)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    sched = lp.lp_schedule()
    sched.team = team
    try:
        with lp.Batch(mats, sched=sched) as b:
            before = b.info()
            with pytest.raises(lp.LPError):
                b.tune(reps=-1)
            b.tune(reps=0)  # the layout step only
            _assert_equal(b.results(), want, "after the layout step")
            assert b.info()["tuned_ms"] == 0
            b.tune(reps=1)
            _assert_equal(b.results(), want, "after the first tune")
            after = b.info()
            assert after["n_resident"] == before["n_resident"] == 20
            b.tune(reps=1)
            for _ in range(3):
                b.run()
            _assert_equal(b.results(), want, "after replays")
            assert b.info()["team_fallbacks"] == 0
    finally:
        for m in mats:
            m.close()


def test_frontier_plan_512_programs_vs_oracle():
    # the same workload by frontier levels: one workgroup per program at a
    # time, the levels its products; results equal the oracle and the matrix-
    # product plan's, on replays of the captured graph and in one call
    progs = gen.batch_programs(0, 512)
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    fr = lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER)
    try:
        with lp.Batch(mats, sched=fr) as b:
            b.run()
            _assert_equal(b.results(), want, "frontier plan")
            ms = b.tune(reps=3)
            assert ms > 0
            for _ in range(3):
                b.run()
            _assert_equal(b.results(), want, "frontier replays")
        _assert_equal(lp.least_model_batch(mats, sched=fr), want, "frontier one call")
    finally:
        for m in mats:
            m.close()


def test_frontier_plan_edge_programs():
    # chains, hubs, facts only, no facts, empty programs, and a program larger
    # than the matrix-product plan's LDS limit
    progs = _edge_programs() + [gen.definite_uniform(4, 300_000, 600_000, 0.02, 4),
                                gen.definite_uniform(7, 500, 900, 0.0, 3),
                                gen.from_rules(3, [(0, []), (1, [0]), (2, [1])])]
    want = _want(progs)
    mats = [lp.Matrix(p) for p in progs]
    try:
        got = lp.least_model_batch(mats, sched=lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER))
        _assert_equal(got, want, "frontier edge programs")
    finally:
        for m in mats:
            m.close()
