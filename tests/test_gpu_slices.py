"""The column-sliced least-model step: the block AND entries laid out in
slices of columns, one pass per slice and product, the slice's part of v in
LDS, a partial AND per row between passes; OR rows and long rows in the last
pass. Forced on small programs with LP_STEP_SLICES_SMALL (slices of 1,024
atoms), and taken by default past what a workgroup's LDS holds. Models and
product counts equal the oracle's (O2) for every step shape and driver."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu

SMALL = lp.LP_STEP_SLICES_SMALL


def _check(p, flags=SMALL, scheds=(None,)):
    want, wp, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p, flags=flags) as m:
        info = m.info
        for s in scheds:
            got, pr = m.least_model(sched=s)
            assert np.array_equal(got, want) and pr == wp, lp.schedule_dict(s) if s is not None else "default"
    return info


def _long_rows_program(seed):
    # block AND rows, AND rows past the block pass's 255 entries, OR rows of
    # many children, facts, and a derivation chain, over 12,000 atoms
    rng = np.random.default_rng(seed)
    n = 12_000
    rules = [(int(a), []) for a in rng.choice(n, 300, replace=False)]
    rules += [(int(h), [int(x) for x in rng.choice(n, int(rng.integers(1, 9)), replace=False)])
              for h in rng.integers(0, n, 20_000)]
    rules += [(int(h), [int(x) for x in rng.choice(n // 3, 300, replace=False)]) for h in rng.integers(0, n, 6)]
    rules += [(7, [int(x)]) for x in rng.integers(0, n, 700)]  # an OR row of 700 children
    rules += [(i, [i - 1]) for i in range(9001, 9400)]
    return gen.from_rules(n, rules)


@pytest.mark.parametrize("seed", range(3))
def test_small_slices_uniform(seed):
    info = _check(gen.definite_uniform(40 + seed, 5000 + 3000 * seed, 12_000 + 5000 * seed, 0.02, 6))
    assert info["n_slices"] >= 5


def test_small_slices_every_step_shape_and_driver():
    p = _long_rows_program(3)
    scheds = [None]
    for w in (4, 8):
        for u in (4, 8, 16):
            scheds.append(lp.make_schedule(variant=lp.LP_STEP_LDS, wpw=w, unroll=u))
            scheds.append(lp.make_schedule(driver=lp.LP_DRIVER_PLAIN, variant=lp.LP_STEP_LDS, wpw=w, unroll=u))
    scheds += [lp.make_schedule(variant=lp.LP_STEP_GLOBAL), lp.make_schedule(driver=lp.LP_DRIVER_PERSISTENT),
               lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER)]
    info = _check(p, scheds=scheds)
    assert info["n_slices"] == 12 and info["n_long_rows"] > 0


def test_small_slices_no_alloc_entry_point():
    p = gen.definite_uniform(50, 9000, 20_000, 0.02, 5)
    want, wp, _, _ = oracle.sd_fixpoint(p)
    with lp.Matrix(p, flags=SMALL) as m:
        got, pr = m.least_model_noalloc()
        assert np.array_equal(got, want) and pr == wp


def test_slices_unsliced_and_tuned_agree():
    p = gen.definite_uniform(60, 6000, 15_000, 0.02, 6)
    with lp.Matrix(p, flags=SMALL) as a, lp.Matrix(p) as b:
        assert a.info["n_slices"] == 6 and b.info["n_slices"] == 0
        ga, pa = a.least_model()
        gb, pb = b.least_model()
        assert np.array_equal(ga, gb) and pa == pb
        ms = a.bench_step(reps=3)
        assert ms > 0


def test_past_the_lds_two_slices_by_default():
    # 2,000,000 atoms: more original atoms than one workgroup's LDS stages
    p = gen.definite_uniform(5, 2_000_000, 4_000_000, 0.01, 4)
    info = _check(p, flags=0, scheds=(None, lp.make_schedule(variant=lp.LP_STEP_GLOBAL),
                                      lp.make_schedule(variant=lp.LP_STEP_LDS, wpw=4, unroll=8)))
    assert info["n_slices"] == 2
