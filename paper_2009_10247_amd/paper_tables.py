"""Programs shaped like the paper's section 4 experiments, solved on the GPU,
with the paper's own sizes and times beside ours for context.

* definite programs at the sizes of the paper's table of definite-program
  results (sparsity 0.99 rows): gen.paper_definite(seed, n, m);
* normal programs at the sizes of its table of normal-program results, with k
  body literals negated: gen.paper_normal(seed, n, m, k);
* transitive closure over random graphs with the |V| and |E| of its table of
  transitive-closure results (the graph data itself is not used):
  gen.transitive_closure(V, edges, grounding="all").

The paper's generator, seeds and graphs are not available, so n' differs; the
paper's times are single-threaded CPU seconds on the hardware it names (an
Intel i7-4770) and are context, not a target. Transitive-closure results are
checked here against a breadth-first closure of the graph; the least and
stable models of the random programs are checked against the CPU oracle in
tests/test_gpu_paper_shapes.py.

* the dense-matrix method on rows of the first two tables, beside the sparse
  engine and the paper's dense and sparse seconds.

    python -m paper_2009_10247_amd.paper_tables [--only definite,normal,tc,dense] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import gen, lp

# (n, m, paper n', paper sparse-matrix seconds)
DEFINITE_ROWS = [
    (1000, 5000, 5788, 0.0071), (1000, 10000, 10799, 0.0127), (1600, 24000, 25198, 0.0357),
    (1600, 30000, 31285, 0.0605), (2000, 36000, 37596, 0.0692), (2000, 40000, 41936, 0.0675),
    (10000, 120000, 127119, 0.3798), (10000, 160000, 167504, 0.4832), (16000, 200000, 211039, 0.8643),
    (16000, 220000, 231439, 0.9429), (20000, 280000, 297293, 0.9048), (20000, 320000, 337056, 1.0614),
]
# (n, m, paper n', k, paper sparse-matrix seconds)
NORMAL_ROWS = [
    (1000, 5000, 6379, 8, 0.0119), (1000, 10000, 12745, 8, 0.0178), (1600, 24000, 30061, 8, 0.0559),
    (1600, 30000, 36402, 7, 0.0832), (2000, 36000, 42039, 5, 0.0897), (2000, 40000, 48187, 8, 0.0991),
    (10000, 120000, 171967, 6, 0.7124), (10000, 160000, 207432, 7, 0.8424), (16000, 200000, 250194, 5, 1.5603),
    (16000, 220000, 278190, 6, 1.8314), (20000, 280000, 357001, 4, 1.9170), (20000, 320000, 396128, 4, 2.1066),
]
# the paper's dense-matrix seconds for the rows it could run (1-6 of both tables)
PAPER_DENSE_S = {
    "definite": {1: 2.0559, 2: 17.9986, 3: 73.3541, 4: 116.1158, 5: 155.4312, 6: 187.6549},
    "normal": {1: 3.9560, 2: 28.1806, 3: 105.4931, 4: 168.8044, 5: 203.2749, 6: 256.9701},
}
# (graph name, |V|, |E|, paper n, paper m, paper n', paper sparse-matrix seconds)
TC_ROWS = [
    ("Club membership", 65, 95, 1200, 14492, 15600, 0.0255), ("Cattle", 28, 217, 1512, 20629, 21924, 0.0365),
    ("Windsurfers", 43, 336, 4324, 99788, 103776, 0.1824), ("Contiguous USA", 49, 107, 4704, 113003, 117600, 0.1830),
    ("Dolphins", 62, 159, 7564, 230861, 238266, 0.4019), ("Train bombing", 64, 243, 8064, 254259, 262080, 0.4524),
    ("Highschool", 70, 366, 9660, 333636, 342930, 0.6618), ("Les Miserables", 77, 254, 11704, 445006, 456456, 0.8300),
]


def _timed(fn, reps):
    out = fn()
    t = time.perf_counter()
    for _ in range(reps):
        out = fn()
    return out, (time.perf_counter() - t) / max(reps, 1)


def closure(V: int, edges) -> np.ndarray:
    """reach[x, y]: y is reachable from x by one or more edges (breadth-first from every x)."""
    adj = [[] for _ in range(V)]
    for x, y in edges:
        adj[x].append(y)
    reach = np.zeros((V, V), dtype=bool)
    for x in range(V):
        frontier = list(adj[x])
        for y in frontier:
            reach[x, y] = True
        while frontier:
            nxt = []
            for z in frontier:
                for y in adj[z]:
                    if not reach[x, y]:
                        reach[x, y] = True
                        nxt.append(y)
            frontier = nxt
    return reach


def run_definite(reps: int, seed: int = 0):
    for i, (n, m, paper_np, paper_s) in enumerate(DEFINITE_ROWS, 1):
        p = gen.paper_definite(seed, n, m)
        t = time.perf_counter()
        mat = lp.Matrix(p)
        build = time.perf_counter() - t
        (model, prods), solve = _timed(lambda: mat.least_model(), reps)
        yield dict(table="definite", row=i, n=n, m=m, n_prime=mat.info["n_rows"], nnz=mat.info["nnz"],
                   paper_n_prime=paper_np, products=prods, least_model_size=int(model.sum()),
                   build_upload_ms=round(build * 1e3, 3), solve_ms=round(solve * 1e3, 3),
                   paper_sparse_s=paper_s)
        mat.close()


def run_normal(reps: int, seed: int = 0):
    for i, (n, m, paper_np, k, paper_s) in enumerate(NORMAL_ROWS, 1):
        p = gen.paper_normal(seed, n, m, k)
        t = time.perf_counter()
        mat = lp.Matrix(p)
        build = time.perf_counter() - t
        r, solve = _timed(lambda: mat.stable_models(), reps)
        yield dict(table="normal", row=i, n=n, m=m, k=k, negated_atoms=mat.info["n_neg"],
                   n_prime=mat.info["n_rows"], nnz=mat.info["nnz"], paper_n_prime=paper_np,
                   products=r["products"], stable_models=r["n_models"],
                   build_upload_ms=round(build * 1e3, 3), solve_ms=round(solve * 1e3, 3), paper_sparse_s=paper_s)
        mat.close()


def run_tc(reps: int, seed: int = 0):
    for i, (name, V, E, paper_n, paper_m, paper_np, paper_s) in enumerate(TC_ROWS, 1):
        edges = gen.random_graph_edges(seed + i, V, E)
        p = gen.transitive_closure(V, edges, grounding="all")
        t = time.perf_counter()
        mat = lp.Matrix(p)
        build = time.perf_counter() - t
        (model, prods), solve = _timed(lambda: mat.least_model(), reps)
        want = closure(V, edges)
        got = model[V * V: 2 * V * V].reshape(V, V).astype(bool)
        yield dict(table="transitive_closure", row=i, graph=f"random ({name}: |V| {V}, |E| {E})", n=p.n_atoms,
                   m=p.n_rules, n_prime=mat.info["n_rows"], nnz=mat.info["nnz"], paper_n=paper_n, paper_m=paper_m,
                   paper_n_prime=paper_np, products=prods, paths=int(got.sum()),
                   closure_matches=bool(np.array_equal(got, want)),
                   build_upload_ms=round(build * 1e3, 3), solve_ms=round(solve * 1e3, 3), paper_sparse_s=paper_s)
        mat.close()


def run_dense(reps: int, seed: int = 0, rows=range(1, 7)):
    """The dense-matrix method (lp_dense_least_model / lp_dense_stable_models) beside the sparse
    engine on rows of the definite- and normal-program tables. The dense matrix of row r holds
    n'^2 bytes (rows 7-12 need 16-157 GB, which one MI355X holds)."""
    for table, spec in (("definite", DEFINITE_ROWS), ("normal", NORMAL_ROWS)):
        for i in rows:
            row = spec[i - 1]
            p = gen.paper_definite(seed, row[0], row[1]) if table == "definite" else \
                gen.paper_normal(seed, row[0], row[1], row[3])
            with lp.Matrix(p) as mat:
                if table == "definite":
                    (_, prods, kern_ms), dense = _timed(lambda: mat.dense_least_model(), max(reps // 2, 1))
                    _, sparse = _timed(lambda: mat.least_model(), reps)
                else:
                    r, dense = _timed(lambda: mat.dense_stable_models(max_models=16), max(reps // 2, 1))
                    prods, kern_ms = r["products"], r["kernel_ms"]
                    _, sparse = _timed(lambda: mat.stable_models(max_models=16), reps)
                yield dict(table=f"dense_{table}", row=i, n=row[0], m=row[1], negated_atoms=mat.info["n_neg"],
                           n_prime=mat.info["n_rows"], products=prods, dense_solve_ms=round(dense * 1e3, 3),
                           dense_product_us=round(kern_ms * 1e3, 1), sparse_solve_ms=round(sparse * 1e3, 3),
                           dense_over_sparse=round(dense / sparse, 1),
                           paper_dense_s=PAPER_DENSE_S[table].get(i),
                           paper_sparse_s=row[3] if table == "definite" else row[4])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="definite,normal,tc",
                    help="comma list of definite, normal, tc, dense")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--dense-rows", default="1-6", help="table rows for the dense method, e.g. 1-6 or 1-12")
    args = ap.parse_args(argv)
    lo, _, hi = args.dense_rows.partition("-")
    dense_rows = range(int(lo), int(hi or lo) + 1)
    runs = {"definite": run_definite, "normal": run_normal, "tc": run_tc,
            "dense": lambda reps: run_dense(reps, rows=dense_rows)}
    ok = True
    for name in args.only.split(","):
        for row in runs[name](args.reps):
            print(json.dumps(row), flush=True)
            ok &= row.get("closure_matches", True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
