"""Python binding of the C-ABI declared in include/lp.h (argument marshalling only).

Every step of the fixpoint runs in liblp.so's HIP kernels; this module only
converts numpy arrays to pointers and status codes to exceptions. There is no
CPU fallback: if liblp.so is missing, loading raises.

Streams may be given as None (default stream), an integer hipStream_t handle,
or any object with a ``cuda_stream`` attribute (a torch.cuda.Stream).

One HIP runtime per process: liblp.so needs libamdhip64.so.7, and PyTorch
ships its own copy under the same soname. When torch is importable, load()
imports it first, so the dynamic linker binds liblp.so to the runtime torch
already mapped and torch's streams and memory are valid handles for the
library; without torch, liblp.so brings the system runtime. load() raises if
two HIP runtimes end up mapped.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblp.so")

LP_OK = 0
LP_E_INVAL = -1
LP_E_NOMEM = -2
LP_E_DEVICE = -3
LP_E_NEGATION = -4
LP_E_TOO_MANY_GUESSES = -5
LP_E_TRUNCATED = -6
LP_E_INTERNAL = -7
LP_E_HOST_ONLY = -8
LP_E_TIMEOUT = -9
LP_MAX_NEG_ATOMS = 24

LP_PRUNE_FACT_GUESSES = 1 << 0
LP_BUILD_HOST_ONLY = 1 << 1
LP_STABLE_FULL_SWEEP = 1 << 2
LP_STABLE_DIRTY_ROWS = 1 << 3
LP_STEP_SLICES_SMALL = 1 << 4

LP_DRIVER_AUTO = 0
LP_DRIVER_PLAIN = 1
LP_DRIVER_BATCHED = 2
LP_DRIVER_PERSISTENT = 3
LP_DRIVER_FRONTIER = 4

LP_STEP_AUTO = 0
LP_STEP_GLOBAL = 1
LP_STEP_LDS = 2

EXPORTS = ("lp_build_matrix", "lp_free_matrix", "lp_matrix_info", "lp_matrix_neg_atoms",
           "lp_matrix_csr", "lp_least_model", "lp_stable_models", "lp_stable_models_guesses",
           "lp_stable_models_search", "lp_least_model_batch", "lp_stable_models_batch",
           "lp_batch_create", "lp_batch_run", "lp_batch_results", "lp_batch_tune",
           "lp_batch_get_info", "lp_batch_free", "lp_matrix_evict", "lp_matrix_upload",
           "lp_server_create", "lp_server_add_program", "lp_server_submit", "lp_server_wait_any",
           "lp_server_take_result", "lp_server_get_stats", "lp_server_free",
           "lp_memory_stats", "lp_release_cached_memory", "lp_bench_spmm",
           "lp_bench_step", "lp_tune_schedule", "lp_set_allocator", "lp_dense_least_model",
           "lp_dense_stable_models", "lp_least_model_noalloc", "lp_schedule_cache_save",
           "lp_schedule_cache_load", "lp_schedule_cache_clear", "lp_schedule_cache_lookup", "lp_last_error")


class LPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lp error {code}: {msg}")
        self.code = code


class lp_info(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_rules", ctypes.c_int32),
                ("n_std_atoms", ctypes.c_int32), ("n_rows", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("n_neg", ctypes.c_int32), ("n_pruned", ctypes.c_int32),
                ("n_and_rows", ctypes.c_int32), ("n_or_rows", ctypes.c_int32),
                ("n_fact_rows", ctypes.c_int32), ("n_empty_rows", ctypes.c_int32),
                ("max_row_len", ctypes.c_int32), ("n_long_rows", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("step_bytes", ctypes.c_int64),
                ("sparsity", ctypes.c_double), ("n_slices", ctypes.c_int32), ("reserved_info", ctypes.c_int32)]


class lp_schedule(ctypes.Structure):
    _fields_ = [("driver", ctypes.c_int32), ("steps_per_sync", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("wpw", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("block", ctypes.c_int32), ("team", ctypes.c_int32), ("team_polls", ctypes.c_int32)]


class lp_batch_info(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("n_resident", ctypes.c_int32),
                ("wpw", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("block", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("step_bytes", ctypes.c_int64), ("tuned_ms", ctypes.c_float),
                ("n_teams", ctypes.c_int32), ("team_members", ctypes.c_int32),
                ("team_fallbacks", ctypes.c_int32)]


class lp_server_config(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("batch_max", ctypes.c_int32),
                ("batch_rows", ctypes.c_int32), ("device", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("tune", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lp_request_info(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_int64), ("program_id", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("status", ctypes.c_int32), ("products", ctypes.c_int32),
                ("n_models", ctypes.c_int64), ("batch_size", ctypes.c_int32), ("built", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class lp_server_stats(ctypes.Structure):
    _fields_ = [("n_programs", ctypes.c_int32), ("n_resident", ctypes.c_int32),
                ("pending", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("batched_requests", ctypes.c_int64), ("alone_requests", ctypes.c_int64),
                ("uploads", ctypes.c_int64), ("evictions", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
                ("peak_used_bytes", ctypes.c_int64), ("hbm_budget", ctypes.c_int64), ("tunes", ctypes.c_int64)]


_lib = None


def hip_runtimes() -> list[str]:
    """Paths of the HIP runtime libraries (libamdhip64) mapped in this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                path = line.split()[-1] if line.count(" ") >= 5 else ""
                if "libamdhip64.so" in os.path.basename(path):
                    found.add(os.path.realpath(path))
    except OSError:
        pass
    return sorted(found)


def load():
    """Load liblp.so (built by paper_2009_10247_amd.build); raise if absent,
    or if the process ends up with two HIP runtimes mapped."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2009_10247_amd.build`")
    try:  # bind to torch's HIP runtime when torch is there (see the module docstring)
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    rts = hip_runtimes()
    if len(rts) > 1:
        raise ImportError("two HIP runtimes are mapped in this process (" + ", ".join(rts) +
                          "); import torch before anything else loads a HIP runtime")
    P = ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "lp_build_matrix": [i32, i32, P, P, P, u32, P, ctypes.POINTER(P)],
        "lp_free_matrix": [P],
        "lp_matrix_info": [P, ctypes.POINTER(lp_info)],
        "lp_matrix_neg_atoms": [P, P],
        "lp_matrix_csr": [P, P, P, P, P],
        "lp_least_model": [P, P, P, P, P],
        "lp_least_model_noalloc": [P, P, P, P],
        "lp_stable_models": [P, P, P, P, i64, P, P, P],
        "lp_stable_models_guesses": [P, P, i64, P, ctypes.POINTER(i64), P, P, i64, P, P],
        "lp_stable_models_search": [P, i64, i32, ctypes.c_uint64, P, i64, ctypes.POINTER(i64), P, P],
        "lp_least_model_batch": [P, i32, P, P, P, P],
        "lp_stable_models_batch": [P, i32, P, P, P, P, P],
        "lp_batch_create": [P, i32, P, P, ctypes.POINTER(P)],
        "lp_batch_run": [P, P],
        "lp_batch_results": [P, P, P, P],
        "lp_batch_tune": [P, i32, ctypes.POINTER(ctypes.c_float), P],
        "lp_batch_get_info": [P, ctypes.POINTER(lp_batch_info)],
        "lp_batch_free": [P],
        "lp_bench_step": [P, P, i32, ctypes.POINTER(ctypes.c_float), P],
        "lp_tune_schedule": [P, i32, ctypes.POINTER(lp_schedule), ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_float), P],
        "lp_set_allocator": [P, P, P],
        "lp_schedule_cache_save": [ctypes.c_char_p],
        "lp_schedule_cache_load": [ctypes.c_char_p],
        "lp_schedule_cache_clear": [],
        "lp_schedule_cache_lookup": [P, ctypes.POINTER(lp_schedule), ctypes.POINTER(i32)],
        "lp_matrix_evict": [P],
        "lp_matrix_upload": [P, P],
        "lp_server_create": [ctypes.POINTER(lp_server_config), ctypes.POINTER(P)],
        "lp_server_add_program": [P, i32, i32, P, P, P, ctypes.POINTER(i32)],
        "lp_server_submit": [P, i32, ctypes.POINTER(i64)],
        "lp_server_wait_any": [P, i32, ctypes.POINTER(lp_request_info)],
        "lp_server_take_result": [P, i64, P, P],
        "lp_server_get_stats": [P, ctypes.POINTER(lp_server_stats)],
        "lp_server_free": [P],
        "lp_memory_stats": [ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "lp_release_cached_memory": [],
        "lp_bench_spmm": [P, i32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32), P],
        "lp_dense_least_model": [P, P, P, P, P],
        "lp_dense_stable_models": [P, P, ctypes.POINTER(i64), P, i64, P, P, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.lp_last_error.argtypes = []
    lib.lp_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _stream(s):
    if s is None:
        return None
    if hasattr(s, "cuda_stream"):
        return ctypes.c_void_p(int(s.cuda_stream))
    return ctypes.c_void_p(int(s))


def _check(rc: int, allow=()):
    if rc != LP_OK and rc not in allow:
        raise LPError(rc, load().lp_last_error().decode())
    return rc


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def make_schedule(driver=LP_DRIVER_AUTO, steps_per_sync=0, variant=LP_STEP_AUTO, grid=0, wpw=0, unroll=0,
                  block=0, team=0, team_polls=0):
    s = lp_schedule()
    s.block = block
    s.team = team
    s.team_polls = team_polls
    s.driver = driver
    s.steps_per_sync = steps_per_sync
    s.variant = variant
    s.grid = grid
    s.wpw = wpw
    s.unroll = unroll
    return s


class Matrix:
    """Program matrix built by lp_build_matrix from a program's three arrays."""

    def __init__(self, prog, flags: int = 0, stream=None):
        lib = load()
        self._head = np.ascontiguousarray(prog.head, dtype=np.int32)
        self._ptr = np.ascontiguousarray(prog.body_ptr, dtype=np.int64)
        self._lit = np.ascontiguousarray(prog.body_lit, dtype=np.int32)
        if self._ptr.shape[0] != self._head.shape[0] + 1:
            raise ValueError("body_ptr must have n_rules + 1 entries")
        self.n_atoms = int(prog.n_atoms)
        self.flags = flags
        h = ctypes.c_void_p()
        _check(lib.lp_build_matrix(self.n_atoms, int(self._head.shape[0]), _ptr(self._head),
                                   self._ptr.ctypes.data, _ptr(self._lit), flags, _stream(stream),
                                   ctypes.byref(h)))
        self._h = h
        # inputs are copied by the library; drop our references
        self._head = self._ptr = self._lit = None
        self.info = self._info()

    def _info(self) -> dict:
        inf = lp_info()
        _check(load().lp_matrix_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in lp_info._fields_}

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _check(load().lp_free_matrix(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def evict(self):
        """Release the device copy (lp_matrix_evict); solves then raise LP_E_HOST_ONLY."""
        _check(load().lp_matrix_evict(self._h))
        self.info = self._info()

    def upload(self, stream=None):
        """Rebuild the device copy from the host CSR (lp_matrix_upload)."""
        _check(load().lp_matrix_upload(self._h, _stream(stream)))
        self.info = self._info()

    def neg_atoms(self) -> np.ndarray:
        out = np.zeros(max(self.info["n_neg"], 1), dtype=np.int32)
        _check(load().lp_matrix_neg_atoms(self._h, out.ctypes.data))
        return out[: self.info["n_neg"]]

    def csr(self):
        """Host copy: (row_ptr int32[n+1], col int32[nnz], kind uint8[n], fact uint8[n])."""
        n, nnz = self.info["n_rows"], self.info["nnz"]
        rp = np.zeros(n + 1, dtype=np.int32)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        kind = np.zeros(max(n, 1), dtype=np.uint8)
        fact = np.zeros(max(n, 1), dtype=np.uint8)
        _check(load().lp_matrix_csr(self._h, rp.ctypes.data, col.ctypes.data, kind.ctypes.data,
                                    fact.ctypes.data))
        return rp, col[:nnz], kind[:n], fact[:n]

    def least_model(self, sched=None, stream=None):
        """(model uint8[n_atoms], products)."""
        model = np.zeros(max(self.n_atoms, 1), dtype=np.uint8)
        prods = ctypes.c_int32(0)
        _check(load().lp_least_model(self._h, model.ctypes.data, ctypes.addressof(prods),
                                     ctypes.byref(sched) if sched is not None else None,
                                     _stream(stream)))
        return model[: self.n_atoms], prods.value

    def least_model_noalloc(self, stream=None):
        """(model uint8[n_atoms], products) by lp_least_model_noalloc (no device allocation)."""
        model = np.zeros(max(self.n_atoms, 1), dtype=np.uint8)
        prods = ctypes.c_int32(0)
        _check(load().lp_least_model_noalloc(self._h, model.ctypes.data, ctypes.addressof(prods), _stream(stream)))
        return model[: self.n_atoms], prods.value

    def stable_models(self, max_models: int = 1024, want_models: bool = True,
                      want_interp: bool = False, stream=None) -> dict:
        """dict(accepted=uint64[W], n_models, models=uint8[m][n_atoms], interp, products, truncated)."""
        K = self.info["n_neg"]
        Wf = max(((1 << K) + 63) // 64, 1)
        acc = np.zeros(Wf, dtype=np.uint64)
        n_models = ctypes.c_int64(0)
        prods = ctypes.c_int32(0)
        models = None
        if want_models:
            # the library writes only the first min(n_models, max_models) rows; the
            # buffer is kept with the matrix (one per thread) and the rows written
            # are copied out
            shape = (max(max_models, 1), max(self.n_atoms, 1))
            tls = self.__dict__.setdefault("_tls", threading.local())
            if getattr(tls, "mbuf", None) is None or tls.mbuf.shape != shape:
                tls.mbuf = np.empty(shape, dtype=np.uint8)
            models = tls.mbuf
        interp = np.zeros((max(self.n_atoms, 1), Wf), dtype=np.uint64) if want_interp else None
        rc = _check(load().lp_stable_models(self._h, acc.ctypes.data, ctypes.addressof(n_models),
                                            models.ctypes.data if models is not None else None,
                                            int(max_models),
                                            interp.ctypes.data if interp is not None else None,
                                            ctypes.addressof(prods), _stream(stream)),
                    allow=(LP_E_TRUNCATED,))
        nm = n_models.value
        out = dict(accepted=acc, n_models=nm, products=prods.value, truncated=rc == LP_E_TRUNCATED)
        if models is not None:
            out["models"] = models[: min(nm, max_models), : self.n_atoms].copy()
        if interp is not None:
            out["interp"] = interp[: self.n_atoms]
        return out

    def dense_least_model(self, stream=None):
        """Algorithm 1 with the dense matrix (lp_dense_least_model): (model uint8[n_atoms], products,
        mean ms of one product launch)."""
        model = np.zeros(max(self.n_atoms, 1), dtype=np.uint8)
        prods = ctypes.c_int32(0)
        ms = ctypes.c_float(0)
        _check(load().lp_dense_least_model(self._h, model.ctypes.data, ctypes.addressof(prods),
                                           ctypes.addressof(ms), _stream(stream)))
        return model[: self.n_atoms], prods.value, ms.value

    def dense_stable_models(self, max_models: int = 1024, want_models: bool = True, stream=None) -> dict:
        """Algorithms 2 and 3 with the dense matrix (lp_dense_stable_models): dict(accepted=uint64[W],
        n_models, models, products, kernel_ms, truncated)."""
        K = self.info["n_neg"]
        Wf = max(((1 << K) + 63) // 64, 1)
        acc = np.zeros(Wf, dtype=np.uint64)
        n_models = ctypes.c_int64(0)
        prods = ctypes.c_int32(0)
        ms = ctypes.c_float(0)
        models = np.zeros((max(max_models, 1), max(self.n_atoms, 1)), dtype=np.uint8) if want_models else None
        rc = _check(load().lp_dense_stable_models(self._h, acc.ctypes.data, ctypes.byref(n_models),
                                                  models.ctypes.data if models is not None else None,
                                                  int(max_models), ctypes.addressof(prods), ctypes.addressof(ms),
                                                  _stream(stream)), allow=(LP_E_TRUNCATED,))
        nm = n_models.value
        out = dict(accepted=acc, n_models=nm, products=prods.value, kernel_ms=ms.value,
                   truncated=rc == LP_E_TRUNCATED)
        if models is not None:
            out["models"] = models[: min(nm, max_models), : self.n_atoms].copy()
        return out

    def bench_step(self, reps: int = 100, sched=None, stream=None) -> float:
        """Average milliseconds of one full-sweep T_P step (HIP events)."""
        ms = ctypes.c_float(0)
        _check(load().lp_bench_step(self._h, ctypes.byref(sched) if sched is not None else None,
                                    int(reps), ctypes.byref(ms), _stream(stream)))
        return ms.value

    def stable_guesses(self, guesses, max_models: int = 0, want_next: bool = True, stream=None) -> dict:
        """Algorithms 2 and 3 on given guesses (lp_stable_models_guesses): dict(accepted=bool[n],
        n_accepted, next=uint64[n] or None, models=uint8[m][n_atoms], products, truncated)."""
        g = np.ascontiguousarray(guesses, dtype=np.uint64)
        n = int(g.shape[0])
        acc = np.zeros(max((n + 63) // 64, 1), dtype=np.uint64)
        na = ctypes.c_int64(0)
        prods = ctypes.c_int32(0)
        nxt = np.zeros(max(n, 1), dtype=np.uint64) if want_next else None
        models = np.zeros((max(max_models, 1), max(self.n_atoms, 1)), dtype=np.uint8) if max_models else None
        rc = _check(load().lp_stable_models_guesses(
            self._h, g.ctypes.data, n, acc.ctypes.data, ctypes.byref(na),
            nxt.ctypes.data if nxt is not None else None, models.ctypes.data if models is not None else None,
            int(max_models), ctypes.addressof(prods), _stream(stream)), allow=(LP_E_TRUNCATED,))
        bits = np.unpackbits(acc.view(np.uint8), bitorder="little")[:n].astype(bool)
        out = dict(accepted=bits, n_accepted=na.value, next=nxt[:n] if nxt is not None else None,
                   products=prods.value, truncated=rc == LP_E_TRUNCATED)
        if models is not None:
            out["models"] = models[: min(na.value, max_models), : self.n_atoms]
        return out

    def stable_search(self, n_samples: int = 4096, rounds: int = 4, seed: int = 0, max_found: int = 1024,
                      want_models: bool = True, stream=None) -> dict:
        """Guess sampling with local search (lp_stable_models_search): dict(found=uint64[k] ascending,
        n_found, models=uint8[k][n_atoms], truncated)."""
        found = np.zeros(max(max_found, 1), dtype=np.uint64)
        nf = ctypes.c_int64(0)
        models = np.zeros((max(max_found, 1), max(self.n_atoms, 1)), dtype=np.uint8) if want_models else None
        rc = _check(load().lp_stable_models_search(
            self._h, int(n_samples), int(rounds), ctypes.c_uint64(seed), found.ctypes.data, int(max_found),
            ctypes.byref(nf), models.ctypes.data if models is not None else None, _stream(stream)),
            allow=(LP_E_TRUNCATED,))
        k = min(nf.value, max_found)
        out = dict(found=found[:k], n_found=nf.value, truncated=rc == LP_E_TRUNCATED)
        if models is not None:
            out["models"] = models[:k, : self.n_atoms]
        return out

    def bench_spmm(self, reps: int = 20, stream=None):
        """(average ms of one stable-model step on the fixpoint, fixpoint products)."""
        ms = ctypes.c_float(0)
        pr = ctypes.c_int32(0)
        _check(load().lp_bench_spmm(self._h, int(reps), ctypes.byref(ms), ctypes.byref(pr), _stream(stream)))
        return ms.value, pr.value

    def tune(self, reps: int = 20, stream=None):
        """(best lp_schedule, step ms, solve ms) from lp_tune_schedule."""
        best = lp_schedule()
        step_ms = ctypes.c_float(0)
        solve_ms = ctypes.c_float(0)
        _check(load().lp_tune_schedule(self._h, int(reps), ctypes.byref(best), ctypes.byref(step_ms),
                                       ctypes.byref(solve_ms), _stream(stream)))
        return best, step_ms.value, solve_ms.value


def schedule_dict(s) -> dict:
    return {name: getattr(s, name) for name, _ in lp_schedule._fields_ if name != "reserved"}


def least_model_batch(mats, sched=None, stream=None):
    """[(model, products)] for a list of Matrix, solved by lp_least_model_batch."""
    n = len(mats)
    outs = [np.zeros(max(m.n_atoms, 1), dtype=np.uint8) for m in mats]
    hs = (ctypes.c_void_p * n)(*[m.handle.value for m in mats])
    ptrs = (ctypes.c_void_p * n)(*[o.ctypes.data for o in outs])
    prods = np.zeros(max(n, 1), dtype=np.int32)
    _check(load().lp_least_model_batch(hs, n, ptrs, prods.ctypes.data,
                                       ctypes.byref(sched) if sched is not None else None,
                                       _stream(stream)))
    return [(outs[i][: mats[i].n_atoms], int(prods[i])) for i in range(n)]


def schedule_cache_save(path: str) -> None:
    """Write the schedule cache (lp_schedule_cache_save)."""
    _check(load().lp_schedule_cache_save(os.fsencode(path)))


def schedule_cache_load(path: str) -> None:
    """Merge a schedule cache file (lp_schedule_cache_load)."""
    _check(load().lp_schedule_cache_load(os.fsencode(path)))


def schedule_cache_clear() -> None:
    _check(load().lp_schedule_cache_clear())


def schedule_cache_lookup(mat):
    """(found, schedule): found 1 with the cached schedule of mat's size bucket, 0 none, 2 the
    default driver solves mat in one workgroup (lp_schedule_cache_lookup)."""
    s = lp_schedule()
    found = ctypes.c_int32(0)
    _check(load().lp_schedule_cache_lookup(mat.handle, ctypes.byref(s), ctypes.byref(found)))
    return found.value, s


def stable_models_batch(mats, stream=None):
    """[dict(accepted=uint64[W], n_models, model=uint8[n_atoms] or None, products)] for a list of
    Matrix, solved by lp_stable_models_batch (the first model of each program)."""
    n = len(mats)
    accs = [np.zeros(max(((1 << m.info["n_neg"]) + 63) // 64, 1), dtype=np.uint64) for m in mats]
    outs = [np.zeros(max(m.n_atoms, 1), dtype=np.uint8) for m in mats]
    hs = (ctypes.c_void_p * max(n, 1))(*[m.handle.value for m in mats])
    aps = (ctypes.c_void_p * max(n, 1))(*[a.ctypes.data for a in accs])
    mps = (ctypes.c_void_p * max(n, 1))(*[o.ctypes.data for o in outs])
    nm = np.zeros(max(n, 1), dtype=np.int64)
    prods = np.zeros(max(n, 1), dtype=np.int32)
    _check(load().lp_stable_models_batch(hs, n, aps, nm.ctypes.data, mps, prods.ctypes.data, _stream(stream)))
    return [dict(accepted=accs[i], n_models=int(nm[i]), products=int(prods[i]),
                 model=outs[i][: mats[i].n_atoms] if nm[i] > 0 else None) for i in range(n)]


class Batch:
    """Batch plan (lp_batch_create) over a list of Matrix; the matrices must
    outlive it. run() enqueues one graph launch; results() reads the last run."""

    def __init__(self, mats, sched=None, stream=None):
        self.mats = list(mats)
        n = len(self.mats)
        hs = (ctypes.c_void_p * max(n, 1))(*[m.handle.value for m in self.mats])
        h = ctypes.c_void_p()
        _check(load().lp_batch_create(hs, n, ctypes.byref(sched) if sched is not None else None,
                                      _stream(stream), ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            load().lp_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, stream=None):
        _check(load().lp_batch_run(self._h, _stream(stream)))

    def results(self, stream=None):
        """[(model uint8[n_atoms], products)] of the last run."""
        n = len(self.mats)
        outs = [np.zeros(max(m.n_atoms, 1), dtype=np.uint8) for m in self.mats]
        ptrs = (ctypes.c_void_p * max(n, 1))(*[o.ctypes.data for o in outs])
        prods = np.zeros(max(n, 1), dtype=np.int32)
        _check(load().lp_batch_results(self._h, ptrs, prods.ctypes.data, _stream(stream)))
        return [(outs[i][: self.mats[i].n_atoms], int(prods[i])) for i in range(n)]

    def tune(self, reps: int = 3, stream=None) -> float:
        ms = ctypes.c_float(0)
        _check(load().lp_batch_tune(self._h, int(reps), ctypes.byref(ms), _stream(stream)))
        return ms.value

    def info(self) -> dict:
        inf = lp_batch_info()
        _check(load().lp_batch_get_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in lp_batch_info._fields_ if name != "reserved"}


def memory_stats() -> dict:
    """Bytes of the library's device pool: held by live objects and cached."""
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load().lp_memory_stats(ctypes.byref(a), ctypes.byref(b)))
    return {"in_use": a.value, "cached": b.value}


def release_cached_memory():
    _check(load().lp_release_cached_memory())


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_hooks = None  # the installed callbacks, kept alive while the library may call them


def set_allocator(alloc=None, release=None):
    """lp_set_allocator with Python callables: alloc(bytes, stream) returns a
    device pointer (int, 0 on failure), release(ptr, stream) frees it; stream
    is the hipStream_t handle as an int (0: the null stream). No arguments:
    the library's own pool again."""
    global _hooks
    if (alloc is None) != (release is None):
        raise ValueError("alloc and release must both be given or both be None")
    if alloc is None:
        _check(load().lp_set_allocator(None, None, None))
        _hooks = None
        return
    a = ALLOC_FN(lambda nbytes, stream, ctx: int(alloc(int(nbytes), int(stream or 0)) or 0))
    r = RELEASE_FN(lambda ptr, stream, ctx: release(int(ptr), int(stream or 0)))
    _check(load().lp_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(r, ctypes.c_void_p), None))
    _hooks = (a, r)


def torch_allocator():
    """(alloc, release) over torch's caching allocator on the current device,
    for set_allocator."""
    import torch

    def alloc(nbytes, stream):
        return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)

    def release(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, release


class Server:
    """Request loop of lp_server_create: register programs, submit requests,
    collect completions (argument marshalling only; the loop is native)."""

    def __init__(self, n_slots=0, batch_max=0, batch_rows=0, hbm_budget=0, device=-1, tune=False):
        cfg = lp_server_config(n_slots=n_slots, batch_max=batch_max, batch_rows=batch_rows, device=device,
                               hbm_budget=int(hbm_budget), tune=1 if tune else 0)
        h = ctypes.c_void_p()
        _check(load().lp_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.n_atoms = {}
        self.n_neg = {}

    def close(self):
        if getattr(self, "_h", None):
            load().lp_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_program(self, prog) -> int:
        head = np.ascontiguousarray(prog.head, dtype=np.int32)
        ptr = np.ascontiguousarray(prog.body_ptr, dtype=np.int64)
        lit = np.ascontiguousarray(prog.body_lit, dtype=np.int32)
        pid = ctypes.c_int32(0)
        _check(load().lp_server_add_program(self._h, int(prog.n_atoms), int(head.shape[0]), _ptr(head),
                                            ptr.ctypes.data, _ptr(lit), ctypes.byref(pid)))
        self.n_atoms[pid.value] = int(prog.n_atoms)
        neg = lit[lit < 0]
        self.n_neg[pid.value] = int(np.unique(neg).shape[0])
        return pid.value

    def submit(self, program_id: int) -> int:
        rid = ctypes.c_int64(0)
        _check(load().lp_server_submit(self._h, int(program_id), ctypes.byref(rid)))
        return rid.value

    def wait_any(self, timeout_ms: int = 1000):
        """Info dict of the next completed request, or None on timeout."""
        inf = lp_request_info()
        rc = _check(load().lp_server_wait_any(self._h, int(timeout_ms), ctypes.byref(inf)), allow=(LP_E_TIMEOUT,))
        if rc == LP_E_TIMEOUT:
            return None
        return {name: getattr(inf, name) for name, _ in lp_request_info._fields_}

    def take_result(self, request_id: int, program_id: int):
        """(model uint8[n_atoms], accepted uint64[ceil(2^K/64)] or None)."""
        n = self.n_atoms[program_id]
        k = self.n_neg[program_id]
        model = np.zeros(max(n, 1), dtype=np.uint8)
        acc = np.zeros(max(((1 << k) + 63) // 64, 1), dtype=np.uint64) if k else None
        _check(load().lp_server_take_result(self._h, int(request_id), model.ctypes.data,
                                            acc.ctypes.data if acc is not None else None))
        return model[:n], acc

    def stats(self) -> dict:
        st = lp_server_stats()
        _check(load().lp_server_get_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in lp_server_stats._fields_}


def unpack_column(interp: np.ndarray, j: int) -> np.ndarray:
    """Column j (one guess) of an interpretation matrix as uint8 per atom."""
    w, b = divmod(int(j), 64)
    return ((interp[:, w] >> np.uint64(b)) & np.uint64(1)).astype(np.uint8)


def accepted_indices(accepted: np.ndarray) -> np.ndarray:
    bits = np.unpackbits(accepted.view(np.uint8), bitorder="little")
    return np.nonzero(bits)[0]
