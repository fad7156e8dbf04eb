"""Host AddressSanitizer / UndefinedBehaviorSanitizer pass over the CPU code:
the matrix builder (csrc/lp_build.cpp) and the oracle (oracle/oracle.c), each
compiled with g++/gcc into a driver of its own (tests/sanitize/), run over
random messy programs (duplicates, shared heads, h <- h, negation), the
paper's examples, edge cases and malformed inputs. Any sanitizer report fails
the test; the drivers' results are compared with the library and the oracle
as normally built."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2009_10247_amd import gen, lp
from tests import _golden

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2009_10247_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in r.stderr.lower() or "cannot find" in r.stderr.lower():
            pytest.skip("no sanitizer runtime for the host compiler: " + r.stderr[-300:])
        raise AssertionError(r.stderr)


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    if not shutil.which("g++") or not shutil.which("gcc"):
        pytest.skip("no host C/C++ compiler")
    d = tmp_path_factory.mktemp("san")
    b = str(d / "builder_san")
    o = str(d / "oracle_san")
    _compile(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", HERE,
              os.path.join(HERE, "builder_main.cpp"), os.path.join(CSRC, "lp_build.cpp"), "-o", b])
    _compile(["gcc", "-std=c11", *SAN, "-I", HERE, os.path.join(HERE, "oracle_main.c"),
              os.path.join(ROOT, "oracle", "oracle.c"), "-o", o])
    return b, o


def _write(path, progs):
    with open(path, "wb") as f:
        for p in progs:
            head = np.ascontiguousarray(p.head, np.int32)
            ptr = np.ascontiguousarray(p.body_ptr, np.int64)
            lit = np.ascontiguousarray(p.body_lit, np.int32)
            f.write(np.array([p.n_atoms, head.shape[0]], np.int32).tobytes())
            f.write(np.array([lit.shape[0]], np.int64).tobytes())
            f.write(head.tobytes() + ptr.tobytes() + lit.tobytes())


def _run(exe, path):
    r = subprocess.run([exe, path], capture_output=True, text=True, env=ENV, timeout=600)
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stderr[-2000:]
    return [ln.split() for ln in r.stdout.splitlines()]


def _malformed():
    P = gen.Program
    i32, i64 = np.int32, np.int64
    return [
        P(2, np.array([0, 9], i32), np.array([0, 1, 2], i64), np.array([1, 0], i32)),     # head out of range
        P(2, np.array([0, -1], i32), np.array([0, 1, 2], i64), np.array([1, 0], i32)),    # negative head
        P(2, np.array([0, 1], i32), np.array([0, 1, 2], i64), np.array([-10, 0], i32)),   # negated atom out of range
        P(2, np.array([0, 1], i32), np.array([0, 1, 2], i64), np.array([5, 0], i32)),     # atom out of range
        P(2, np.array([0, 1], i32), np.array([1, 1, 2], i64), np.array([1, 0], i32)),     # body_ptr[0] != 0
        P(2, np.array([0, 1], i32), np.array([0, 2, 1], i64), np.array([1, 0], i32)),     # body_ptr decreasing
        P(-1, np.zeros(0, i32), np.zeros(1, i64), np.zeros(0, i32)),                      # negative atom count
    ]


def _valid():
    progs = [gen.tiny_random(s, max_atoms=16, max_rules=40, max_body=4,
                             p_neg=0.0 if s % 2 else 0.3) for s in range(400)]
    progs += [_golden.program(_golden.load(n)) for n in ("example1.txt", "example2.txt")]
    progs += [gen.even_loops(4), gen.odd_loop(), gen.definite_uniform(1, 300, 700, 0.05, 4),
              gen.normal_uniform(2, 200, 400, 4, k_neg=6, p_neg=0.3),
              gen.Program(0, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32)),
              gen.from_rules(3, [(0, [0]), (1, [1, 1, 0]), (2, [gen.neg(2)]), (2, [2, gen.neg(2)])]),
              gen.from_rules(5, [(4, [])] * 5 + [(3, [4, 4, 4])])]
    return progs


def test_builder_under_sanitizers(drivers, tmp_path):
    valid, bad = _valid(), _malformed()
    path = str(tmp_path / "progs.bin")
    _write(path, valid + bad)
    out = _run(drivers[0], path)
    assert len(out) == len(valid) + len(bad)
    for p, row in zip(valid, out):
        assert row[0] == "0" and row[6] == "0", row
        with lp.Matrix(p, flags=lp.LP_BUILD_HOST_ONLY) as m:
            assert [int(row[1]), int(row[2]), int(row[3])] == [m.info["n_rows"], m.info["nnz"], m.info["n_neg"]]
        with lp.Matrix(p, flags=lp.LP_BUILD_HOST_ONLY | lp.LP_PRUNE_FACT_GUESSES) as m:
            assert int(row[10]) == m.info["n_pruned"]
    for row in out[len(valid):]:
        assert row == [str(lp.LP_E_INVAL)] * 2, row


def test_oracle_under_sanitizers(drivers, tmp_path):
    valid, bad = _valid(), _malformed()
    path = str(tmp_path / "progs.bin")
    _write(path, valid + bad)
    out = _run(drivers[1], path)
    assert len(out) == len(valid) + len(bad)
    for p, row in zip(valid, out):
        K = int(row[0])
        if K == 0:
            lm, prods, _, _ = oracle.sd_fixpoint(p)
            assert row[1] == "0" and row[3] == "0", row
            assert int(row[2]) == int(lm.sum()) and int(row[4]) == prods
        else:
            ref = oracle.stable(p)
            assert row[1] == "0", row
            assert int(row[2]) == int(ref["accept"].sum()) and int(row[3]) == ref["products"]
            assert int(row[4]) == int(row[2])  # every accepted model passes the GL check
    for row in out[len(valid):]:
        assert int(row[0]) < 0, row
