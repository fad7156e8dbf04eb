"""Parity of the HIP engine (through the C-ABI) with the CPU oracle.

Every comparison is exact: models, product counts, accepted-guess masks and
per-guess fixpoints are integers and bit sets."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2009_10247_amd import gen, lp
from tests import _golden

pytestmark = pytest.mark.gpu


def _least(prog, **kw):
    with lp.Matrix(prog) as m:
        return m.least_model(**kw)


def _check_least(prog, sched=None):
    want, want_prods, n_std, _ = oracle.sd_fixpoint(prog)
    got, prods = _least(prog, sched=sched)
    assert np.array_equal(got, want)
    assert prods == want_prods
    assert np.array_equal(want, oracle.least_model(prog))
    return prods


# ---------------------------------------------------------------- least models

def test_example1_on_gpu():
    d = _golden.load("example1.txt")
    got, prods = _least(_golden.program(d))
    assert [a for a, x in zip(d["atoms"], got) if x] == d["least_model"]
    assert prods == d["products"][0]


SCHEDULES = {
    "plain-global": lp.make_schedule(driver=lp.LP_DRIVER_PLAIN, variant=lp.LP_STEP_GLOBAL),
    "plain-lds": lp.make_schedule(driver=lp.LP_DRIVER_PLAIN, variant=lp.LP_STEP_LDS),
    "batched-global": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, steps_per_sync=3, variant=lp.LP_STEP_GLOBAL),
    "batched-lds-grid3": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, steps_per_sync=5, variant=lp.LP_STEP_LDS,
                                          grid=3),
    "persistent": lp.make_schedule(driver=lp.LP_DRIVER_PERSISTENT),
    "persistent-grid2": lp.make_schedule(driver=lp.LP_DRIVER_PERSISTENT, grid=2),
    "persistent-w8-u16": lp.make_schedule(driver=lp.LP_DRIVER_PERSISTENT, wpw=8, unroll=16),
    "lds-w4-u4": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, variant=lp.LP_STEP_LDS, wpw=4, unroll=4),
    "lds-w4-u16": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, variant=lp.LP_STEP_LDS, wpw=4, unroll=16),
    "lds-w8-u16": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, variant=lp.LP_STEP_LDS, wpw=8, unroll=16),
    "global-w4-u16": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, variant=lp.LP_STEP_GLOBAL, wpw=4, unroll=16),
    "global-w8-u4": lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, variant=lp.LP_STEP_GLOBAL, wpw=8, unroll=4,
                                     grid=5),
    "frontier": lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER),
    "auto": None,
}


@pytest.mark.parametrize("name", list(SCHEDULES))
def test_tiny_programs_match_oracle(name):
    sched = SCHEDULES[name]
    for seed in range(150):
        p = gen.tiny_random(seed, max_atoms=16, max_rules=40, max_body=4)
        got, prods = _least(p, sched=sched)
        assert brute.from_vector(got) == brute.least_model(p), seed
        assert prods == oracle.sd_fixpoint(p)[1], seed


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_definite_1k_atoms_2k_rules(seed):
    _check_least(gen.definite_uniform(seed, 1000, 2000, 0.05, 4))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 257, 4097])
def test_ragged_sizes(n):
    _check_least(gen.definite_uniform(n, n, 3 * n, 0.05, 4))


def test_empty_and_factless_programs():
    empty = gen.Program(0, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32))
    got, prods = _least(empty)
    assert got.shape == (0,) and prods == 1
    p = gen.definite_uniform(4, 500, 1000, 0.0, 4)
    got, prods = _least(p)
    assert got.sum() == 0 and prods == 1
    rule_free = gen.Program(7, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32))
    got, prods = _least(rule_free)
    assert got.sum() == 0 and prods == 1


@pytest.mark.parametrize("name", list(SCHEDULES))
def test_long_or_and_rows_split_in_segments(name):
    # one head with 10,000 rules: an OR row of 10,000 entries (3 segments);
    # one rule with a 9,000-atom body: a split AND row (3 segments) that fires;
    # a second split AND row that must not fire (one body atom never true).
    rng = np.random.default_rng(7)
    n = 20_000
    rules = [(a, []) for a in range(0, 12_000)]
    rules += [(19_000, [int(x)]) for x in rng.integers(12_000, 18_000, size=10_000)]
    rules += [(19_001, list(range(0, 9_000)))]
    rules += [(19_002, list(range(1, 9_000)) + [19_500])]
    rules += [(int(h), [int(b)]) for h, b in zip(rng.integers(12_000, 18_000, 3000), rng.integers(0, 12_000, 3000))]
    rules += [(19_003, [19_001, 19_000])]
    p = gen.from_rules(n, rules)
    with lp.Matrix(p) as m:
        assert m.info["n_long_rows"] >= 3
    _check_least(p, sched=SCHEDULES[name])


@pytest.mark.parametrize("L", [1, 2, 100, 1000])
def test_chain_products(L):
    p = gen.from_rules(L, [(0, [])] + [(i, [i - 1]) for i in range(1, L)])
    assert _check_least(p) == L


@pytest.mark.parametrize("name", list(SCHEDULES))
def test_chain_zipf_scaled(name):
    p = gen.chain_zipf(1, n_atoms=100_000, n_rules=500_000, chain_len=300)
    assert _check_least(p, sched=SCHEDULES[name]) == 300


@pytest.mark.slow
def test_chain_zipf_full_size():
    # 1,000,000 atoms, 5,000,000 rules, 2,000-long chain: the benchmarked workload
    p = gen.chain_zipf(0)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    assert want_prods == 2000
    with lp.Matrix(p) as m:
        for name in ("batched-global", "persistent", "auto", "lds-w4-u16", "lds-w8-u16"):
            got, prods = m.least_model(sched=SCHEDULES[name])
            assert np.array_equal(got, want) and prods == 2000, name
        # the schedule the benchmark times: the autotuner's choice
        best, _, _ = m.tune(reps=3)
        got, prods = m.least_model(sched=best)
        assert np.array_equal(got, want) and prods == 2000, lp.schedule_dict(best)


@pytest.mark.parametrize("variant", ["lds", "global"])
def test_more_atoms_than_lds_holds(variant):
    # 1,400,000 atoms: more original atoms than one workgroup's LDS can stage
    # (about 1.29 million), so the staged step gathers the rest from global
    # memory (the mixed form)
    p = gen.definite_uniform(11, 1_400_000, 2_000_000, 0.01, 4)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    v = lp.LP_STEP_LDS if variant == "lds" else lp.LP_STEP_GLOBAL
    for shape in ((8, 16), (4, 8)):
        got, prods = _least(p, sched=lp.make_schedule(driver=lp.LP_DRIVER_BATCHED, variant=v, wpw=shape[0],
                                                      unroll=shape[1]))
        assert np.array_equal(got, want) and prods == want_prods, shape


def test_bench_step_runs():
    p = gen.chain_zipf(2, n_atoms=50_000, n_rules=250_000, chain_len=50)
    with lp.Matrix(p) as m:
        for v in (lp.LP_STEP_GLOBAL, lp.LP_STEP_LDS):
            ms = m.bench_step(reps=20, sched=lp.make_schedule(variant=v))
            assert ms > 0
        # the step leaves the matrix usable and the answer unchanged
        got, prods = m.least_model()
    assert np.array_equal(got, oracle.least_model(p)) and prods == 50


def test_tuned_schedule_gives_the_same_model():
    p = gen.chain_zipf(3, n_atoms=60_000, n_rules=300_000, chain_len=40)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        best, step_ms, solve_ms = m.tune(reps=3)
        assert step_ms > 0 and solve_ms > 0
        assert best.driver in (lp.LP_DRIVER_BATCHED, lp.LP_DRIVER_PERSISTENT)
        got, prods = m.least_model(sched=best)
    assert np.array_equal(got, want) and prods == want_prods


def test_bench_and_tune_small_program_with_default_schedule():
    # the default driver solves small programs in one workgroup and keeps only
    # the model's bits; timing steps needs a whole interpretation, which the
    # step benchmark and the autotuner take from the batched driver
    p = gen.definite_uniform(0, 1000, 2000, 0.05, 4)
    want, want_prods, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p) as m:
        assert m.bench_step(reps=5) > 0
        best, step_ms, solve_ms = m.tune(reps=2)
        assert step_ms > 0 and solve_ms > 0
        for sched in (None, best):
            got, prods = m.least_model(sched=sched)
            assert np.array_equal(got, want) and prods == want_prods


def test_unsupported_shape_is_an_error():
    with lp.Matrix(gen.definite_uniform(0, 100, 200)) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model(sched=lp.make_schedule(wpw=3))
        assert e.value.code == lp.LP_E_INVAL
        with pytest.raises(lp.LPError) as e:
            m.least_model(sched=lp.make_schedule(wpw=16))
        assert e.value.code == lp.LP_E_INVAL


def test_concurrent_matrices_do_not_interfere():
    progs = [gen.definite_uniform(s, 2000, 5000, 0.03, 4) for s in range(6)]
    mats = [lp.Matrix(p) for p in progs]
    try:
        res = [m.least_model() for m in mats]
        res_again = [m.least_model() for m in reversed(mats)][::-1]
        for p, (g, pr), (g2, pr2) in zip(progs, res, res_again):
            want, wp, _, _ = oracle.sd_fixpoint(p)
            assert np.array_equal(g, want) and pr == wp
            assert np.array_equal(g2, want) and pr2 == wp
    finally:
        for m in mats:
            m.close()


def test_default_driver_concurrent_solves_of_one_matrix():
    # small programs take the one-workgroup LDS loop under the default driver;
    # its descriptor and result buffers are per call, so one matrix solved from
    # several threads on their own streams gives the oracle's result every time
    import threading

    import torch

    progs = [gen.definite_uniform(40 + s, 1500 + 400 * s, 3000 + 800 * s, 0.03, 4) for s in range(3)]
    want = [oracle.sd_fixpoint(p)[:2] for p in progs]
    mats = [lp.Matrix(p) for p in progs]
    streams = [torch.cuda.Stream() for _ in range(4)]  # non-default streams of the one HIP runtime
    errors, done = [], []

    def worker(k):
        try:
            for it in range(20):
                i = (k + it) % len(mats)
                g, pr = mats[i].least_model(stream=streams[k])
                if not (np.array_equal(g, want[i][0]) and pr == want[i][1]):
                    errors.append((k, it, i))
                done.append(k)
        except BaseException as e:  # noqa: BLE001
            errors.append(repr(e))

    try:
        threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert errors == [] and len(done) == 4 * 20
    finally:
        for m in mats:
            m.close()


def test_batch_entry_point_equals_single_solves():
    progs = gen.batch_programs(11, count=24, lo=100, hi=5000)
    mats = [lp.Matrix(p) for p in progs]
    try:
        out = lp.least_model_batch(mats)
        for p, (g, pr) in zip(progs, out):
            want, wp, _, _ = oracle.sd_fixpoint(p)
            assert np.array_equal(g, want) and pr == wp
    finally:
        for m in mats:
            m.close()


def test_negation_rejected_by_least_model():
    p = gen.from_rules(2, [(0, [gen.neg(1)])])
    with lp.Matrix(p) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model()
        assert e.value.code == lp.LP_E_NEGATION


# ---------------------------------------------------------------- stable models

def _check_stable(prog, flags=0, want_interp=True, threads=0):
    res_o = oracle.stable(prog, threads=threads, want_interp=want_interp and flags == 0)
    with lp.Matrix(prog, flags=flags) as m:
        res = m.stable_models(max_models=4096, want_interp=want_interp and flags == 0)
    K = res_o["neg_atoms"].shape[0]
    acc_o = np.nonzero(res_o["accept"])[0]
    assert np.array_equal(lp.accepted_indices(res["accepted"]), acc_o)
    assert res["n_models"] == acc_o.shape[0]
    if want_interp and flags == 0:
        assert np.array_equal(res["interp"], res_o["interp"])
        assert res["products"] == res_o["products"]
    for i, j in enumerate(acc_o[: res["models"].shape[0]]):
        w, b = divmod(int(j), 64)
        col = ((res_o["interp"][:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8) \
            if res_o["interp"] is not None else None
        if col is not None:
            assert np.array_equal(res["models"][i], col)
        assert oracle.gl_check(prog, res["models"][i])
    return res


def test_example2_on_gpu():
    d = _golden.load("example2.txt")
    p = _golden.program(d)
    res = _check_stable(p)
    assert [[a for a, x in zip(d["atoms"], mdl) if x] for mdl in res["models"]] == [["t"]]
    for flags in (0, lp.LP_PRUNE_FACT_GUESSES):
        with lp.Matrix(p, flags=flags) as m:
            r = m.stable_models()
            assert list(lp.accepted_indices(r["accepted"])) == d["accepted_guesses"]


def test_tiny_normal_programs_match_brute_force():
    for seed in range(120):
        p = gen.tiny_random(40_000 + seed, max_atoms=9, max_rules=16, max_body=3, p_neg=0.35)
        res = _check_stable(p)
        got = sorted(brute.from_vector(m) for m in res["models"])
        assert got == brute.stable_models(p), seed
        with lp.Matrix(p, flags=lp.LP_STABLE_DIRTY_ROWS) as m:
            dirty = m.stable_models(max_models=4096)
        assert np.array_equal(dirty["accepted"], res["accepted"]) and dirty["products"] == res["products"], seed


@pytest.mark.parametrize("k", [1, 3, 5, 6, 7, 9, 12])
def test_normal_programs_each_guess_width(k):
    _check_stable(gen.normal_uniform(k, 600, 1200, 5, k_neg=k, p_neg=0.2))


@pytest.mark.parametrize("n", [1, 4, 8])
def test_even_loops(n):
    res = _check_stable(gen.even_loops(n))
    assert res["n_models"] == 2 ** n


def test_even_loops_16_atoms_negated_without_oracle():
    # 8 even loops: K = 16, 65,536 guesses, exactly 256 models, each picking
    # exactly one atom per loop
    p = gen.even_loops(8)
    with lp.Matrix(p) as m:
        res = m.stable_models(max_models=1000)
    assert res["n_models"] == 256
    mods = res["models"]
    assert mods.shape == (256, 16)
    assert np.all(mods[:, 0::2] + mods[:, 1::2] == 1)
    assert len({bytes(r) for r in mods}) == 256


def test_odd_loop_and_definite():
    with lp.Matrix(gen.odd_loop()) as m:
        assert m.stable_models()["n_models"] == 0
    p = gen.definite_uniform(3, 400, 800)
    with lp.Matrix(p) as m:
        res = m.stable_models(want_interp=True)
    assert res["n_models"] == 1 and np.array_equal(res["models"][0], oracle.least_model(p))


def test_pruning_keeps_the_stable_models():
    for seed in range(30):
        base = gen.normal_uniform(seed, 200, 400, 4, k_neg=6, p_neg=0.3)
        rng = np.random.default_rng(seed)
        negs = oracle.negated_atoms(base)
        facts = [(int(q), []) for q in rng.choice(negs, size=2, replace=False)]
        p = gen.from_rules(base.n_atoms, list(base.rules()) + facts)
        _check_stable(p, flags=lp.LP_PRUNE_FACT_GUESSES, want_interp=False)
        with lp.Matrix(p, flags=lp.LP_PRUNE_FACT_GUESSES) as m:
            assert m.info["n_pruned"] == 2
            with pytest.raises(lp.LPError) as e:
                m.stable_models(want_interp=True)
            assert e.value.code == lp.LP_E_INVAL


def test_truncation_reports_all_models():
    with lp.Matrix(gen.even_loops(5)) as m:
        res = m.stable_models(max_models=7)
    assert res["truncated"] and res["n_models"] == 32 and res["models"].shape[0] == 7


@pytest.mark.parametrize("k", [1, 3, 6, 7, 9, 12])
def test_stable_dirty_rows_equal_full_sweep(k):
    # products by dirty rows (LP_STABLE_DIRTY_ROWS; the default only from 2^19
    # row-words) and full sweeps (LP_STABLE_FULL_SWEEP): the same fixpoint
    # matrix, product count and models, equal to the oracle's
    p = gen.normal_uniform(100 + k, 800, 1600, 5, k_neg=k, p_neg=0.25)
    ref = oracle.stable(p, want_interp=True)
    out = {}
    for flags in (lp.LP_STABLE_DIRTY_ROWS, lp.LP_STABLE_FULL_SWEEP):
        with lp.Matrix(p, flags=flags) as m:
            out[flags] = m.stable_models(max_models=4096, want_interp=True)
    a, b = out[lp.LP_STABLE_DIRTY_ROWS], out[lp.LP_STABLE_FULL_SWEEP]
    assert np.array_equal(a["interp"], b["interp"]) and np.array_equal(a["interp"], ref["interp"])
    assert a["products"] == b["products"] == ref["products"]
    assert np.array_equal(a["accepted"], b["accepted"]) and np.array_equal(a["models"], b["models"])


def test_stable_dirty_rows_chain_and_loops():
    # a long derivation chain through negation-free rows (many products, one
    # row changing per product) and even loops (many models)
    rules = [(0, [gen.neg(1)]), (1, [gen.neg(0)])] + [(i, [i - 1]) for i in range(2, 400)]
    for p in (gen.from_rules(400, rules), gen.even_loops(6)):
        ref = oracle.stable(p, want_interp=True)
        with lp.Matrix(p, flags=lp.LP_STABLE_DIRTY_ROWS) as m:
            res = m.stable_models(max_models=4096, want_interp=True)
        assert np.array_equal(res["interp"], ref["interp"]) and res["products"] == ref["products"]


def test_normal_10k_atoms_16_negated_full_width():
    # 10,000 atoms, 20,000 rules, 16 negated atoms: all 65,536 guesses, every
    # per-guess fixpoint compared with the oracle (products by dirty rows), and
    # the full-sweep products giving the same matrix
    p = gen.normal_uniform(0)
    res = _check_stable(p, threads=16)
    with lp.Matrix(p, flags=lp.LP_STABLE_FULL_SWEEP) as m:
        full = m.stable_models(max_models=4096, want_interp=True)
    assert np.array_equal(full["interp"], res["interp"]) and full["products"] == res["products"]
