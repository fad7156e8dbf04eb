"""The library beside PyTorch: one HIP runtime in the process, torch streams
accepted by every solve entry point, and device memory taken from torch's
caching allocator through lp_set_allocator. Results are compared with the
CPU oracle."""
import gc

import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp

pytestmark = pytest.mark.gpu


def _programs():
    small = gen.definite_uniform(71, 1000, 2000, 0.05, 4)          # one-workgroup LDS loop
    large = gen.definite_uniform(72, 120_000, 240_000, 0.02, 4)   # batched step driver
    normal = gen.normal_uniform(73, 400, 800, 4, k_neg=8, p_neg=0.2)
    return small, large, normal


def _check_least(m, p, stream):
    want, wp, _, _ = oracle.sd_fixpoint(p)
    got, pr = m.least_model(stream=stream)
    assert np.array_equal(got, want) and pr == wp


def _check_stable(m, p, stream):
    ref = oracle.stable(p, want_interp=True)
    res = m.stable_models(want_interp=True, stream=stream)
    assert np.array_equal(lp.accepted_indices(res["accepted"]), np.nonzero(ref["accept"])[0])
    assert np.array_equal(res["interp"], ref["interp"])
    assert res["products"] == ref["products"]


def test_one_hip_runtime_in_the_process():
    import torch

    lp.load()
    assert torch.cuda.is_available()
    assert len(lp.hip_runtimes()) == 1, lp.hip_runtimes()


def test_torch_streams_through_every_solve_entry_point():
    import torch

    small, large, normal = _programs()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    assert s1.cuda_stream != 0 and s2.cuda_stream != 0
    with lp.Matrix(small, stream=s1) as ms, lp.Matrix(large, stream=s2) as ml, \
            lp.Matrix(normal, stream=s1) as mn:
        _check_least(ms, small, s2)
        _check_least(ml, large, s1)
        _check_stable(mn, normal, s2)
        progs = gen.batch_programs(74, count=12, lo=200, hi=4000)
        mats = [lp.Matrix(p, stream=s2) for p in progs]
        try:
            with lp.Batch(mats, stream=s1) as b:
                for _ in range(2):
                    b.run(stream=s1)
                    for p, (g, pr) in zip(progs, b.results(stream=s1)):
                        want, wp, _, _ = oracle.sd_fixpoint(p)
                        assert np.array_equal(g, want) and pr == wp
            for p, (g, pr) in zip(progs, lp.least_model_batch(mats, stream=s2)):
                want, wp, _, _ = oracle.sd_fixpoint(p)
                assert np.array_equal(g, want) and pr == wp
        finally:
            for m in mats:
                m.close()
    torch.cuda.synchronize()


def test_allocations_go_through_torch_caching_allocator():
    import torch

    gc.collect()
    lp.load()
    base = lp.memory_stats()
    assert base["in_use"] == 0, "library pool blocks still live from an earlier test"
    alloc, release = lp.torch_allocator()
    live, counts = {}, {"alloc": 0, "release": 0}

    def counting_alloc(nbytes, stream):
        ptr = alloc(nbytes, stream)
        if ptr:
            live[ptr] = nbytes
            counts["alloc"] += 1
        return ptr

    def counting_release(ptr, stream):
        assert ptr in live, "release of a block the hook did not allocate"
        del live[ptr]
        counts["release"] += 1
        release(ptr, stream)

    small, large, normal = _programs()
    stream = torch.cuda.Stream()
    torch_before = torch.cuda.memory_allocated()
    lp.set_allocator(counting_alloc, counting_release)
    try:
        ms = lp.Matrix(small, stream=stream)
        ml = lp.Matrix(large, stream=stream)
        mn = lp.Matrix(normal, stream=stream)
        assert live and torch.cuda.memory_allocated() > torch_before
        # the installed hook stays while its blocks are live
        with pytest.raises(lp.LPError) as e:
            lp.set_allocator()
        assert e.value.code == lp.LP_E_INVAL
        _check_least(ms, small, stream)
        _check_least(ml, large, stream)
        _check_stable(mn, normal, stream)
        progs = gen.batch_programs(75, count=8, lo=200, hi=3000)
        mats = [lp.Matrix(p, stream=stream) for p in progs]
        for p, (g, pr) in zip(progs, lp.least_model_batch(mats, stream=stream)):
            want, wp, _, _ = oracle.sd_fixpoint(p)
            assert np.array_equal(g, want) and pr == wp
        # nothing went to the library's own pool
        assert lp.memory_stats()["in_use"] == 0
        for m in [ms, ml, mn, *mats]:
            m.close()
        assert live == {} and counts["alloc"] == counts["release"] > 0
    finally:
        gc.collect()
        lp.set_allocator()
    assert torch.cuda.memory_allocated() == torch_before
    # the pool serves again once the hook is removed
    with lp.Matrix(small) as m:
        _check_least(m, small, None)
        assert lp.memory_stats()["in_use"] > 0
