"""CPU oracle for least and stable models (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package. The engine never does.

* ``least_model``   -- O1, Dowling-Gallier forward chaining on P (oracle.c)
* ``sd_fixpoint``   -- O2, synchronous stage count on the standardized program
* ``stable``        -- O3, per-guess least models of P+ plus the consistency test
* ``gl_check``      -- O4, Gelfond-Lifschitz reduct test
* ``brute``         -- O5, exhaustive enumeration for programs of <= 16 atoms
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-result", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        common = [i32, i32, P, P, P]
        lib.orc_least_model.argtypes = common + [P]
        lib.orc_sd_fixpoint.argtypes = common + [P, P, P, P]
        lib.orc_stable.argtypes = common + [i64, i64, i32, P, P, P]
        lib.orc_gl_check.argtypes = common + [P]
        lib.orc_negated_atoms.argtypes = common + [P, P]
        for f in (lib.orc_least_model, lib.orc_sd_fixpoint, lib.orc_stable, lib.orc_gl_check,
                  lib.orc_negated_atoms):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned {code}")
        self.code = code


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _args(prog):
    head = np.ascontiguousarray(prog.head, dtype=np.int32)
    ptr = np.ascontiguousarray(prog.body_ptr, dtype=np.int64)
    lit = np.ascontiguousarray(prog.body_lit, dtype=np.int32)
    keep = (head, ptr, lit)
    return keep, [int(prog.n_atoms), int(head.shape[0]), _ptr(head), ptr.ctypes.data, _ptr(lit)]


def _check(rc):
    if rc < 0:
        raise OracleError(rc)
    return rc


def least_model(prog) -> np.ndarray:
    """O1: uint8[n_atoms], 1 for atoms of LM(P)."""
    keep, a = _args(prog)
    out = np.zeros(max(prog.n_atoms, 1), dtype=np.uint8)
    _check(_load().orc_least_model(*a, out.ctypes.data))
    return out[:prog.n_atoms]


def sd_fixpoint(prog):
    """O2: (model uint8[n_atoms], products, |B_{P^delta}|, |LM(P^delta)|)."""
    keep, a = _args(prog)
    out = np.zeros(max(prog.n_atoms, 1), dtype=np.uint8)
    prods = ctypes.c_int32(0)
    nstd = ctypes.c_int32(0)
    ntrue = ctypes.c_int64(0)
    _check(_load().orc_sd_fixpoint(*a, out.ctypes.data, ctypes.addressof(prods),
                                   ctypes.addressof(nstd), ctypes.addressof(ntrue)))
    return out[:prog.n_atoms], prods.value, nstd.value, ntrue.value


def negated_atoms(prog) -> np.ndarray:
    keep, a = _args(prog)
    out = np.zeros(max(prog.n_atoms, 1), dtype=np.int32)
    k = ctypes.c_int32(0)
    _check(_load().orc_negated_atoms(*a, out.ctypes.data, ctypes.addressof(k)))
    return out[:k.value].copy()


def stable(prog, guess_begin: int = 0, guess_count: int | None = None, threads: int = 0,
           want_interp: bool = False):
    """O3 over guesses [guess_begin, guess_begin + guess_count).

    Returns dict(accept=uint8[count], interp=uint64[n_atoms][W] or None,
    products=int, neg_atoms=int32[K]).
    """
    K = negated_atoms(prog).shape[0]
    if guess_count is None:
        guess_count = (1 << K) - guess_begin
    keep, a = _args(prog)
    acc = np.zeros(max(guess_count, 1), dtype=np.uint8)
    W = (guess_count + 63) // 64
    interp = np.zeros((prog.n_atoms, W), dtype=np.uint64) if want_interp else None
    prods = ctypes.c_int32(0)
    _check(_load().orc_stable(*a, int(guess_begin), int(guess_count), int(threads), acc.ctypes.data,
                              interp.ctypes.data if (interp is not None and interp.size) else None,
                              ctypes.addressof(prods)))
    return dict(accept=acc[:guess_count], interp=interp, products=prods.value,
                neg_atoms=negated_atoms(prog))


def stable_models(prog, threads: int = 0):
    """All stable models as a list of uint8[n_atoms] vectors in guess order."""
    res = stable(prog, threads=threads, want_interp=True)
    models = []
    for j in np.nonzero(res["accept"])[0]:
        w, b = divmod(int(j), 64)
        models.append(((res["interp"][:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8))
    return models, res


def gl_check(prog, interp) -> bool:
    """O4: True iff interp is a stable model (Gelfond-Lifschitz)."""
    keep, a = _args(prog)
    v = np.ascontiguousarray(interp, dtype=np.uint8)
    return bool(_check(_load().orc_gl_check(*a, v.ctypes.data)))
