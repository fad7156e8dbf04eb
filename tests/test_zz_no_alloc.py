"""lp_least_model_noalloc through the C-ABI: the same models and product
counts as lp_least_model, on two calls in a row (the second with a smaller
program), with the library's device pool untouched; oversized matrices are
refused before any device work."""
import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu


def _same(a, b):
    return np.array_equal(a[0], b[0]) and a[1] == b[1]


def test_noalloc_equals_least_model_larger_then_smaller():
    import torch

    big = gen.chain_zipf(91, n_atoms=200_000, n_rules=1_000_000)  # step driver: 2,000 products, long OR rows
    mid = gen.definite_uniform(92, 60_000, 120_000, 0.02, 5)        # step driver
    small = gen.definite_uniform(93, 1000, 2000, 0.05, 4)           # one-workgroup LDS loop
    stream = torch.cuda.Stream()
    with lp.Matrix(big) as mb, lp.Matrix(mid) as mm, lp.Matrix(small) as ms:
        want = [m.least_model(stream=stream) for m in (mb, mm, ms)]
        for p, w in zip((big, mid, small), want):
            lm, prods, _, _ = oracle.sd_fixpoint(p)
            assert np.array_equal(w[0], lm) and w[1] == prods
        info = [m._info() for m in (mb, mm, ms)]
        pool = lp.memory_stats()
        # two calls in a row, the second smaller; then the other orders
        for order in ((0, 1), (1, 2), (0, 2), (2, 0), (0, 1, 2, 1, 0)):
            for k in order:
                got = (mb, mm, ms)[k].least_model_noalloc(stream=stream if k != 1 else None)
                assert _same(got, want[k]), (order, k)
        assert lp.memory_stats() == pool  # no pool allocation, no pool release
        assert [m._info() for m in (mb, mm, ms)] == info  # nothing attached to the matrices
    torch.cuda.synchronize()


def test_noalloc_refuses_matrices_past_its_region():
    # 17,000,000 atoms (one fact): two bit-packed interpretations take 4.25 MB
    p = gen.from_rules(17_000_000, [(0, [])])
    with lp.Matrix(p) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model_noalloc()
        assert e.value.code == lp.LP_E_INVAL and "scratch" in str(e.value)
        g, pr = m.least_model()
        assert g[0] == 1 and g[1:].sum() == 0 and pr == 1


def test_noalloc_argument_errors():
    with lp.Matrix(gen.from_rules(2, [(0, [gen.neg(1)])])) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model_noalloc()
        assert e.value.code == lp.LP_E_NEGATION
    with lp.Matrix(gen.definite_uniform(0, 50, 100), flags=lp.LP_BUILD_HOST_ONLY) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model_noalloc()
        assert e.value.code == lp.LP_E_HOST_ONLY
