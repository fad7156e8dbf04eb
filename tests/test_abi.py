"""CPU tests of the C-ABI library: it loads, exports what include/lp.h
declares, and its host-side matrix builder reproduces the paper's worked
examples and the standardization's closed forms. No compute call is made."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp
from tests import _golden

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = lp.load()
    names = _declared()
    assert set(names) == set(lp.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_no_cpu_fallback_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(lp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lp, "_lib", None)
    with pytest.raises(ImportError):
        lp.load()


def _host(prog, flags=0):
    return lp.Matrix(prog, flags=flags | lp.LP_BUILD_HOST_ONLY)


def _value_matrix(m):
    """Dense matrix of Definitions 2/7 rebuilt from CSR + row kinds."""
    rp, col, kind, fact = m.csr()
    n = rp.shape[0] - 1
    M = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        cols = col[rp[i]:rp[i + 1]]
        for c in cols:
            M[i][c] = Fraction(1, len(cols)) if kind[i] else Fraction(1)
    return M


def test_example1_csr_matches_example4():
    d = _golden.load("example1.txt")
    with _host(_golden.program(d)) as m:
        rp, col, kind, fact = m.csr()
        assert list(rp) == d["csr_row_index"]
        assert list(col) == d["csr_col_index"]
        M = _value_matrix(m)
        vals = [float(M[i][c]) for i in range(7) for c in col[rp[i]:rp[i + 1]]]
        assert vals == d["csr_value"]
        # COO of Example 3
        rows = [i for i in range(7) for _ in range(rp[i + 1] - rp[i])]
        assert rows == d["coo_row"] and list(col) == d["coo_col"]
        # the printed 7x7 matrix
        for i, name in enumerate(d["std_atoms"]):
            assert M[i] == d["matrix"][name], name
        assert list(fact) == [0, 0, 0, 1, 1, 0, 0]
        assert m.info["n_std_atoms"] == 7 and m.info["n_rows"] == 7


def test_example2_matrix():
    d = _golden.load("example2.txt")
    with _host(_golden.program(d)) as m:
        assert m.info["n_neg"] == 1 and m.info["n_rows"] == 7
        assert list(m.neg_atoms()) == [d["atoms"].index("t")]
        M = _value_matrix(m)
        for i, name in enumerate(d["std_atoms"]):
            assert M[i] == d["matrix"][name], name


def _closed_form(prog):
    """N_d = N + sum of k_h over heads with k_h >= 2; nnz from the rule bodies."""
    n = prog.n_atoms
    k = np.bincount(prog.head, minlength=n)
    n_new = int(k[k >= 2].sum())
    negs = sorted({-l - 1 for l in prog.body_lit.tolist() if l < 0})
    nnz = 0
    for h, body in prog.rules():
        nnz += len(set(body)) if body else 1
    nnz += n_new + len(negs)
    return n + n_new, n + n_new + len(negs), nnz


@pytest.mark.parametrize("seed", range(12))
def test_closed_form_sizes(seed):
    progs = [gen.definite_uniform(seed, 300, 700, 0.05, 4),
             gen.tiny_random(seed, 16, 40, 4, p_neg=0.2),
             gen.normal_uniform(seed, 400, 800, 5, k_neg=6)]
    for p in progs:
        n_std, n_rows, nnz = _closed_form(p)
        with _host(p) as m:
            assert (m.info["n_std_atoms"], m.info["n_rows"], m.info["nnz"]) == (n_std, n_rows, nnz)
            rp, col, kind, fact = m.csr()
            assert np.all(np.diff(rp) >= 0) and rp[-1] == nnz
            for i in range(m.info["n_rows"]):
                seg = col[rp[i]:rp[i + 1]]
                assert np.all(np.diff(seg) > 0)  # sorted, deduped
        if (p.body_lit >= 0).all():
            assert oracle.sd_fixpoint(p)[2] == n_std  # the oracle's own rewrite agrees


def test_row_kinds_equal_exact_theta():
    # count == len  <=>  sum of len copies of 1/len >= 1, in exact rationals
    for L in range(1, 40):
        for c in range(0, L + 1):
            assert (c == L) == (Fraction(c, L) >= 1)


def test_sd_rows_group_children_consecutively():
    p = gen.definite_uniform(5, 200, 600, 0.05, 3)
    with _host(p) as m:
        rp, col, kind, fact = m.csr()
        for a in range(p.n_atoms):
            if kind[a] == 0 and rp[a + 1] > rp[a]:
                seg = col[rp[a]:rp[a + 1]]
                assert np.array_equal(seg, np.arange(seg[0], seg[0] + seg.shape[0]))


def test_prune_flag_counts_fact_negations():
    rules = [(0, []), (1, [gen.neg(0)]), (2, [gen.neg(3)]), (3, [gen.neg(2)])]
    p = gen.from_rules(4, rules)
    with _host(p, lp.LP_PRUNE_FACT_GUESSES) as m:
        assert m.info["n_neg"] == 3 and m.info["n_pruned"] == 1


@pytest.mark.parametrize("bad", ["head", "lit", "ptr0", "ptrdec"])
def test_malformed_programs_are_rejected(bad):
    head = np.array([0, 1], np.int32)
    ptr = np.array([0, 1, 2], np.int64)
    lit = np.array([1, 0], np.int32)
    if bad == "head":
        head[1] = 9
    elif bad == "lit":
        lit[0] = -10
    elif bad == "ptr0":
        ptr[0] = 1
    elif bad == "ptrdec":
        ptr = np.array([0, 2, 1], np.int64)
    with pytest.raises(lp.LPError) as e:
        _host(gen.Program(2, head, ptr, lit))
    assert e.value.code == lp.LP_E_INVAL


def test_host_only_matrix_refuses_solves():
    with _host(gen.definite_uniform(0, 50, 100)) as m:
        with pytest.raises(lp.LPError) as e:
            m.least_model()
        assert e.value.code == lp.LP_E_HOST_ONLY


def test_empty_program_builds():
    with _host(gen.Program(0, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32))) as m:
        assert m.info["n_rows"] == 0 and m.info["nnz"] == 0


def test_build_flags_leave_no_packed_fp32_in_device_code(tmp_path):
    # the library is built with build.NO_PACKED_FP32; on a float2 kernel that
    # hipcc -O3 otherwise compiles to v_pk_add_f32, the flags remove it
    import subprocess

    from paper_2009_10247_amd import build

    src = tmp_path / "pk.hip"
    src.write_text("#include <hip/hip_runtime.h>\n"
                   "__global__ void k(float2 *a, const float2 *b, int n) {\n"
                   "  int i = blockIdx.x * blockDim.x + threadIdx.x;\n"
                   "  if (i < n) { float2 x = a[i], y = b[i]; x.x += y.x; x.y += y.y; a[i] = x; }\n}\n")

    def device_asm(extra):
        out = tmp_path / "pk.s"
        subprocess.check_call([build.hipcc(), "-O3", f"--offload-arch={build.ARCH}", "--offload-device-only",
                               "-S", *extra, "-o", str(out), str(src)], stderr=subprocess.DEVNULL)
        return out.read_text()

    assert "v_pk_add_f32" in device_asm([])
    assert not re.search(r"v_pk_(add|mul|fma)_f32", device_asm(build.NO_PACKED_FP32))
    assert all(f in build.command("x.so") for f in build.NO_PACKED_FP32)
