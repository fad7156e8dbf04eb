#!/usr/bin/env python3
"""Benchmark of the T_P fixpoint engine on one MI355X.

A step is one least-model solve (Algorithm 1: initial vector, synchronous
theta(M v) products until nothing changes, model copied out) of a synthetic
definite program with 1,000,000 atoms, 5,000,000 rules (bodies of 1-8 atoms,
1% facts, Zipf(1.1) heads) and an embedded 2,000-long derivation chain, so
each solve performs 2,000 full-matrix products. The program matrix is built
and resident in HBM before the timed region.

value = rule-body entries processed per second = nnz * products / seconds.

Also reported: the dominant kernel (one full-sweep T_P step) against the HBM
roofline, the CPU oracle timed on this host, stable-model guesses/s on a
normal program with 10,000 atoms, 20,000 rules and 16 negated atoms, and 512
programs of 1e3-1e5 atoms solved by one batch launch against 512 sequential
single-program solves, and the dense-matrix method (the paper's third method)
beside the sparse engine on the same programs.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_bytes(info: dict) -> int:
    """Algorithmic bytes of one full-sweep step on the device layout the
    kernel reads (lp_info.step_bytes): the per-word metadata, the 8-bit AND
    lengths, the AND column entries, the OR child-range table, the long-row
    segments, one read of v and one write of u (bit-packed)."""
    return int(info["step_bytes"])


def recorded_traffic(kernel: str, step_bytes_now: int, source: str = "lp_step.hip"):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (2 x FETCH_SIZE + WRITE_SIZE, calibrated against a known-size copy), or
    None when no record matches the current kernel source (`source` under
    csrc/) and bytes per launch."""
    import glob
    import hashlib
    import re

    src = os.path.join(ROOT, "paper_2009_10247_amd", "csrc", source)
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if not line.startswith("traffic-record:"):
                continue
            m = re.match(r'traffic-record: kernel="([^"]+)" source_sha1=(\w+) step_bytes=(\d+) .*'
                         r'bytes_per_launch=(\d+)', line.strip())
            if m and m.group(1) == kernel and m.group(2) == sha and int(m.group(3)) == step_bytes_now:
                return int(m.group(4))
    return None


def step_mode(info: dict, sched) -> int:
    """Form of the step kernel the library launches: 0 gathers from global
    memory, 1 all of v staged in LDS (the original atoms fit in the 160 KB of a
    workgroup beside the ballot slots), 3 column-sliced (one pass per slice of
    the original atoms, past what one workgroup's LDS holds)."""
    from paper_2009_10247_amd import lp
    if sched.variant == lp.LP_STEP_GLOBAL:
        return 0
    if info.get("n_slices", 0) > 0:
        return 3
    cap_words = 163840 // 8 - 16 * (sched.unroll + 1) - 2
    return 1 if (info["n_atoms"] + 63) // 64 <= cap_words else 2


def csr_step_bytes(info: dict) -> int:
    """The same step on a plain int32 CSR (row pointers, column indices,
    row-kind bits, v and u bit-packed): what a CSR kernel would move."""
    n, nnz = info["n_rows"], info["nnz"]
    return 4 * (n + 1) + 4 * nnz + 3 * ((n + 7) // 8)


def bench_small(gen, lp, stream) -> dict:
    """The 1,000-atom definite program (2,000 rules, 5% facts, bodies 1-4): a
    solve is about 15 products of a 45 KB layout, so it is bound by launch and
    memory latency, not bandwidth. Wall-clock microseconds per solve (model in
    host memory) with the default driver, the persistent driver, and a
    one-program batch plan (the whole loop in one workgroup's LDS)."""
    import numpy as np

    p = gen.definite_uniform(0, 1000, 2000, 0.05, 4)
    out = {"workload": "definite_uniform: 1,000 atoms, 2,000 rules, 5% facts, bodies 1-4", "unit": "us per solve"}
    with lp.Matrix(p, stream=stream) as m:
        ref = m.least_model(stream=stream)
        out["n_rows"] = m.info["n_rows"]
        out["products"] = ref[1]
        reps = 50
        for name, sched in (("default", None), ("persistent", lp.make_schedule(driver=lp.LP_DRIVER_PERSISTENT))):
            m.least_model(sched=sched, stream=stream)
            t = time.perf_counter()
            for _ in range(reps):
                r = m.least_model(sched=sched, stream=stream)
            out[name] = round((time.perf_counter() - t) * 1e6 / reps, 1)
            assert np.array_equal(r[0], ref[0]) and r[1] == ref[1]
        with lp.Batch([m], stream=stream) as plan:
            plan.run(stream=stream)
            plan.results(stream=stream)
            t = time.perf_counter()
            for _ in range(reps):
                plan.run(stream=stream)
                r = plan.results(stream=stream)[0]
            out["batch_plan"] = round((time.perf_counter() - t) * 1e6 / reps, 1)
            assert np.array_equal(r[0], ref[0]) and r[1] == ref[1]
    log(f"[bench] small program: {out}")
    return out


def cpu_threads() -> int:
    """Host threads the oracle baselines use: OMP_NUM_THREADS if set, else all CPUs."""
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return max(1, os.cpu_count() or 1)


def bench_batch(args, torch, gen, lp, stream) -> dict:
    """Many programs at once: 512 definite programs (atoms log-uniform in
    1e3..1e5, 2x rules, bodies 1..6, 2% facts) solved by one launch of the
    batch kernel (a replay of the plan's hipGraph, shape autotuned first),
    against the same 512 solved one after another by the plain driver (one
    launch and one host read of the change count per product) and by the
    library's default driver."""
    t = time.perf_counter()
    progs = gen.batch_programs(args.seed, 512)
    mats = [lp.Matrix(p, stream=stream) for p in progs]
    log(f"[bench] batch: 512 programs generated and built in {time.perf_counter() - t:.1f}s")
    try:
        plan = lp.Batch(mats, stream=stream)
        tuned_ms = plan.tune(reps=3, stream=stream)
        binfo = plan.info()
        plan.run(stream=stream)
        res = plan.results(stream=stream)
        torch.cuda.synchronize()
        reps = max(5, args.steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.run(stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        dev_ms = e0.elapsed_time(e1) / reps
        t = time.perf_counter()
        for _ in range(reps):
            plan.run(stream=stream)
            res2 = plan.results(stream=stream)
        e2e_ms = (time.perf_counter() - t) * 1e3 / reps
        plain = lp.make_schedule(driver=lp.LP_DRIVER_PLAIN)
        seq = {}
        for name, sched in (("plain", plain), ("default", None)):
            for mm in mats[:8]:  # warm the step kernels
                mm.least_model(sched=sched, stream=stream)
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = [mm.least_model(sched=sched, stream=stream) for mm in mats]
            seq[name] = (time.perf_counter() - t) * 1e3
            for (g, pr), (g2, pr2) in zip(res, out):
                assert pr == pr2 and (g == g2).all(), "batch result differs from the single-program solve"
        for (g, pr), (g2, pr2) in zip(res, res2):
            assert pr == pr2 and (g == g2).all()
        # the same 512 programs by frontier levels (semi-naive: each entry visited once per solve
        # rather than once per product), one launch of a frontier plan
        fplan = lp.Batch(mats, sched=lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER), stream=stream)
        fplan.run(stream=stream)
        fres = fplan.results(stream=stream)
        for (g, pr), (g2, pr2) in zip(res, fres):
            assert pr == pr2 and (g == g2).all(), "frontier plan differs from the matrix-product plan"
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(reps):
            fplan.run(stream=stream)
        f1.record(stream)
        torch.cuda.synchronize()
        frontier_ms = f0.elapsed_time(f1) / reps
        fplan.close()
        prods = [pr for _, pr in res]
        entries = sum(mm.info["nnz"] * pr for mm, pr in zip(mats, prods))
        layout = sum((mm.info["step_bytes"] - 2 * ((mm.info["n_rows"] + 7) // 8)) * pr
                     for mm, pr in zip(mats, prods))
        # roofline of the batch launch: the int32-CSR bytes of every product of
        # every program (4 (N'+1) + 4 nnz + 3 N'/8 each), per launch
        csr = sum(csr_step_bytes(mm.info) * pr for mm, pr in zip(mats, prods))
        achieved = csr / (dev_ms / 1e3) / 1e9
        kname = f"tp_batch_kernel<{binfo['wpw']}, {binfo['unroll']}>"
        traffic = recorded_traffic(kname, csr, "lp_batch.hip")
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                    "bytes_per_launch": csr, "bytes": "algorithmic: int32 CSR, 4 (N'+1) + 4 nnz + 3 N'/8 "
                    "bytes per product of each program, summed over the batch",
                    "traffic_over_bytes": round(traffic / csr, 4) if traffic else None}
        out = {"workload": "512 definite programs, atoms log-uniform 1e3-1e5, rules 2x atoms, bodies 1-6, "
                           "2% facts; one launch of the batch kernel (graph replay)",
               "programs": 512, "atoms": sum(p.n_atoms for p in progs), "nnz": binfo["nnz"],
               "products_total": int(sum(prods)), "products_max": int(max(prods)),
               "ms_per_batch": round(dev_ms, 3), "ms_per_batch_with_results": round(e2e_ms, 3),
               "entries_per_s": round(entries / (dev_ms / 1e3), 1),
               "layout_GB/s": round(layout / (dev_ms / 1e3) / 1e9, 1), "roofline": roofline,
               "frontier_ms_per_batch": round(frontier_ms, 3),
               "sequential_plain_ms": round(seq["plain"], 3), "sequential_default_ms": round(seq["default"], 3),
               "speedup_vs_sequential_plain": round(seq["plain"] / e2e_ms, 2),
               "speedup_vs_sequential_default": round(seq["default"] / e2e_ms, 2),
               "shape": {k: binfo[k] for k in ("wpw", "unroll", "block", "grid", "lds_bytes")},
               "teams": {k: binfo[k] for k in ("n_teams", "team_members", "team_fallbacks")},
               "tuned_ms": round(tuned_ms, 3)}
        if not args.no_cpu_baseline:
            # the oracle's forward chaining per program: one thread on a sample of 128 programs
            # (scaled to 512), and every program over a pool of host threads
            import oracle
            from concurrent.futures import ThreadPoolExecutor

            t = time.perf_counter()
            for p in progs[:128]:
                oracle.sd_fixpoint(p)
            one = (time.perf_counter() - t) * 512 / 128
            thr = cpu_threads()
            t = time.perf_counter()
            with ThreadPoolExecutor(thr) as ex:
                ores = list(ex.map(oracle.sd_fixpoint, progs))
            alls = time.perf_counter() - t
            for (g, pr), o in zip(res, ores):
                assert pr == o[1] and (g == o[0]).all(), "batch result differs from the oracle"
            out["cpu_baseline"] = {"kind": "oracle", "unit": "ms per 512 programs",
                                   "one_thread": {"value": round(one * 1e3, 1), "cores": 1,
                                                  "sample": "programs 0-127 in generation order, scaled to 512"},
                                   "all_cores": {"value": round(alls * 1e3, 1), "cores": thr,
                                                 "sample": "all 512 programs, one per host thread at a time"}}
        log(f"[bench] batch: {out}")
        plan.close()
        return out
    finally:
        for mm in mats:
            mm.close()


def copy_probe(torch, dev, stream, mib: int = 1024) -> float:
    """Device-to-device copy bandwidth (bytes read + written per second, in
    GB/s) of a mib-MiB buffer: the bandwidth a plain streaming kernel reaches
    on this GPU, beside the published peak."""
    src = torch.ones((mib << 20) // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            dst.copy_(src)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * (mib << 20) / (ms / 1e3) / 1e9


MFMA_INT8_PEAK_TOPS = 5000.0


def dense_roofline(n_rows: int, columns: int, ms: float) -> dict:
    """Roofline of one dense product: the method reads every one of the n'^2
    matrix entries (one byte each) and reads and writes n' bytes per column;
    a product with c columns is 2 n'^2 c int8 operations. The bound is the
    larger of the two times at peak (HBM 8 TB/s, int8 matrix cores 5.0 POP/s)."""
    ops = 2.0 * n_rows * n_rows * columns
    nbytes = float(n_rows) * n_rows + 2.0 * n_rows * columns
    secs = ms / 1e3
    if columns > 1 and ops / (MFMA_INT8_PEAK_TOPS * 1e12) >= nbytes / (HBM_PEAK_GBS * 1e9):
        ach = ops / secs / 1e12
        return {"bound": "mfma", "achieved": round(ach, 1), "peak": MFMA_INT8_PEAK_TOPS, "unit": "TOP/s",
                "frac": round(ach / MFMA_INT8_PEAK_TOPS, 4), "ops_per_launch": ops}
    ach = nbytes / secs / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": nbytes}


def bench_dense(gen, lp, stream) -> dict:
    """The dense-matrix method against the sparse engine on the same programs:
    the sixth rows of the paper's definite- and normal-program tables (2,000
    atoms, 40,000 rules; the normal one with 8 negated body literals), and the
    normal program with 16 negated atoms (65,536 guess columns), where the
    dense product is bound by the matrix cores."""
    import numpy as np

    from paper_2009_10247_amd import paper_tables as pt

    out = {}
    cases = (("definite_2k_40k", gen.paper_definite(0, 2000, 40000), False, ("definite", 6)),
             ("normal_2k_40k_k8", gen.paper_normal(0, 2000, 40000, 8), True, ("normal", 6)),
             ("normal_10k_k16", gen.normal_uniform(0), True, None))
    for name, p, stable, paper in cases:
        with lp.Matrix(p, stream=stream) as m:
            n = m.info["n_rows"]
            K = m.info["n_neg"]
            # first call warms up; the second is timed (solve includes building the dense matrix)
            if stable:
                m.dense_stable_models(max_models=16, stream=stream)
                t = time.perf_counter()
                r = m.dense_stable_models(max_models=16, stream=stream)
                dense_s = time.perf_counter() - t
                prods, kms = r["products"], r["kernel_ms"]
                m.stable_models(max_models=16, stream=stream)
                t = time.perf_counter()
                rs = m.stable_models(max_models=16, stream=stream)
                sparse_s = time.perf_counter() - t
                assert np.array_equal(r["accepted"], rs["accepted"]) and r["products"] == rs["products"]
                cols = 1 << K
            else:
                m.dense_least_model(stream=stream)
                t = time.perf_counter()
                model, prods, kms = m.dense_least_model(stream=stream)
                dense_s = time.perf_counter() - t
                m.least_model(stream=stream)
                t = time.perf_counter()
                smodel, sprods = m.least_model(stream=stream)
                sparse_s = time.perf_counter() - t
                assert np.array_equal(model, smodel) and prods == sprods
                cols = 1
        kern = "dense_gemm_kernel" if stable else "dense_gemv_kernel"
        row = {"n_rows": n, "negated_atoms": K, "columns": cols, "products": prods,
               "dense_solve_ms": round(dense_s * 1e3, 3), "sparse_solve_ms": round(sparse_s * 1e3, 3),
               "dense_over_sparse": round(dense_s / sparse_s, 1), "kernel": kern,
               "us_per_launch": round(kms * 1e3, 2), "roofline": dense_roofline(n, cols, kms)}
        if paper:
            row["paper_dense_s"] = pt.PAPER_DENSE_S[paper[0]][paper[1]]
            spec = (pt.DEFINITE_ROWS if paper[0] == "definite" else pt.NORMAL_ROWS)[paper[1] - 1]
            row["paper_sparse_s"] = spec[3] if paper[0] == "definite" else spec[4]
        out[name] = row
        log(f"[bench] dense {name}: {row}")
    return out


def bench_serving(args, gen, lp) -> dict:
    """The serving configuration: a pool of 256 programs (atoms log-uniform
    1e3-1e6, rules 3x atoms, bodies 1-6, 2% facts, K ~ U{0..12} negated atoms;
    K = 0 a least-model query, else a stable-model query), Zipf(1.0)
    popularity, Poisson arrivals at each rate through the native request loop.
    Every pool program is solved alone first, and every streamed result must
    equal its alone result byte for byte."""
    from paper_2009_10247_amd import serve

    t = time.perf_counter()
    pool = gen.serving_pool(args.seed, 256, 1e3, 1e6, max_k=12)
    rates = [float(x) for x in args.serve_rates.split(",")]
    log(f"[bench] serving pool generated in {time.perf_counter() - t:.1f}s")
    rows = []
    with lp.Server(n_slots=args.serve_slots) as srv:
        t = time.perf_counter()
        pids = [srv.add_program(p) for p in pool]
        ref = serve.solve_alone(srv, pids)
        log(f"[bench] serving: registered and solved alone in {time.perf_counter() - t:.1f}s")
        w = serve.zipf_weights(len(pids))
        for k, rate in enumerate(rates):
            row = serve.run_stream(srv, pids, w, rate, args.serve_requests, args.seed + 1 + k, ref)
            assert row["mismatches"] == 0, f"{row['mismatches']} streamed results differ from alone"
            rows.append({f: row[f] for f in ("rate", "requests", "least", "stable", "p50_ms", "p99_ms",
                                             "mean_ms", "p99_queue_ms", "completed_per_s", "entries_per_s",
                                             "batched", "batched_stable", "mismatches")})
            log(f"[bench] serving {rows[-1]}")
        st = srv.stats()
    return {"workload": "serving pool: 256 programs, atoms log-uniform 1e3-1e6, rules 3x atoms, bodies 1-6, "
                        "2% facts, K ~ U{0..12}; Zipf(1.0) popularity, Poisson arrivals",
            "slots": args.serve_slots, "rates": rows,
            "uploads": st["uploads"], "evictions": st["evictions"], "batches": st["batches"],
            "peak_used_bytes": st["peak_used_bytes"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--step-reps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stable", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-frontier", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-rates", default="100,1000,3000")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--dense-only", action="store_true",
                    help="run only the dense-matrix contrast and print its JSON")
    ap.add_argument("--cpu-budget-s", type=float, default=12.0)
    ap.add_argument("--sweep", action="store_true", help="time every step shape (diagnostic)")
    ap.add_argument("--tune-reps", type=int, default=20)
    ap.add_argument("--schedule", default="",
                    help="skip the tuner: variant,wpw,unroll[,driver] e.g. lds,2,16,batched")
    ap.add_argument("--step-only", action="store_true",
                    help="only time the step kernel of --schedule (for hardware-counter runs)")
    ap.add_argument("--scale-rules", type=int, default=1,
                    help="multiply the program's rules (4: a layout larger than the 256 MB Infinity "
                         "Cache, so the stream comes from DRAM)")
    ap.add_argument("--scale-atoms", type=int, default=1,
                    help="multiply the program's atoms (past about 1.29 million original atoms the "
                         "staged step gathers the rest from global memory)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="with --step-only: also run one device-to-device copy of this many MiB, a "
                         "known-size kernel that calibrates the byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design, not a measured configuration.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2009_10247_amd import gen, lp

    torch.cuda.init()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    if args.dense_only:
        print(json.dumps(bench_dense(gen, lp, stream)), flush=True)
        return 0

    t = time.perf_counter()
    n_atoms, n_rules = 1_000_000 * args.scale_atoms, 5_000_000 * args.scale_rules
    prog = gen.chain_zipf(args.seed, n_atoms=n_atoms, n_rules=n_rules)
    log(f"[bench] generated chain_zipf seed={args.seed}: {n_atoms} atoms, {prog.n_rules} rules, "
        f"{prog.n_literals} literals in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    m = lp.Matrix(prog, stream=stream)
    build_s = time.perf_counter() - t
    info = m.info
    log(f"[bench] matrix: N'={info['n_rows']} nnz={info['nnz']} long rows={info['n_long_rows']} "
        f"build {build_s:.2f}s")
    if args.schedule:
        f = args.schedule.split(",")
        sched = lp.make_schedule(variant={"lds": lp.LP_STEP_LDS, "global": lp.LP_STEP_GLOBAL}[f[0]],
                                 wpw=int(f[1]), unroll=int(f[2]), steps_per_sync=64,
                                 driver={"batched": lp.LP_DRIVER_BATCHED, "persistent": lp.LP_DRIVER_PERSISTENT,
                                         "plain": lp.LP_DRIVER_PLAIN}[f[3] if len(f) > 3 else "batched"])
        if args.step_only:
            step_sched = lp.make_schedule(variant=sched.variant, wpw=sched.wpw, unroll=sched.unroll)
            ms = m.bench_step(reps=args.step_reps, sched=step_sched, stream=stream)
            log(f"[bench] step-only {args.schedule}: {ms * 1e3:.2f} us/launch, "
                f"{step_bytes(info) / (ms / 1e3) / 1e9:.0f} GB/s")
            if args.copy_mb:
                n = args.copy_mb << 20
                src = torch.ones(n // 4, dtype=torch.int32, device=dev)
                dst = torch.empty_like(src)
                torch.cuda.synchronize()
                dst.copy_(src)
                torch.cuda.synchronize()
                log(f"[bench] copied {args.copy_mb} MiB device-to-device")
            return 0
    else:
        # autotune outside the timed region (step shape and driver)
        t = time.perf_counter()
        sched, tune_step_ms, tune_solve_ms = m.tune(reps=args.tune_reps, stream=stream)
        log(f"[bench] tuned in {time.perf_counter() - t:.1f}s: {lp.schedule_dict(sched)} "
            f"step {tune_step_ms * 1e3:.1f} us, solve {tune_solve_ms:.2f} ms")

    for i in range(args.warmup):
        model, products = m.least_model(sched=sched, stream=stream)
        log(f"[bench] warmup {i}: products={products} |LM|={int(model.sum())}")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    prods = []
    marks = []
    for i in range(args.steps):
        model, products = m.least_model(sched=sched, stream=stream)
        prods.append(products)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(stream)
        marks.append(ev)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    ms_per_step = ev_ms / max(args.steps, 1)
    per_solve = [(e0 if i == 0 else marks[i - 1]).elapsed_time(marks[i]) for i in range(len(marks))]
    products = prods[-1]
    assert all(p == products for p in prods)
    entries = info["nnz"] * products
    value = entries / (ms_per_step / 1e3)
    log(f"[bench] {args.steps} solves: {ms_per_step:.3f} ms/solve (events), wall {wall * 1e3 / args.steps:.3f} ms, "
        f"products={products}, {ms_per_step * 1e3 / products:.2f} us/product")

    B = step_bytes(info)
    variants = {}
    if args.sweep:
        for v, vname in ((lp.LP_STEP_LDS, "lds"), (lp.LP_STEP_GLOBAL, "global")):
            for w in (4, 8):
                for u in (4, 8, 16):
                    ms = m.bench_step(reps=args.step_reps, stream=stream,
                                      sched=lp.make_schedule(variant=v, wpw=w, unroll=u))
                    variants[f"{vname}-w{w}-u{u}"] = round(ms * 1e3, 2)
        log(f"[bench] step us per shape: {variants}")

    # dominant kernel, timed with HIP events around its launches inside the library
    if sched.driver == lp.LP_DRIVER_PERSISTENT:
        kern_ms = m.bench_step(reps=max(3, args.steps), sched=sched, stream=stream)
        Bl = B * products
        kname = f"tp_fixpoint_persistent_kernel<{sched.wpw}, {sched.unroll}>"
    else:
        step_sched = lp.make_schedule(variant=sched.variant, wpw=sched.wpw, unroll=sched.unroll, grid=sched.grid)
        kern_ms = m.bench_step(reps=args.step_reps, sched=step_sched, stream=stream)
        Bl = B
        kname = f"tp_step_kernel<{step_mode(info, sched)}, {sched.wpw}, {sched.unroll}>"
    # achieved: the algorithmic bytes of a full step on the int32 CSR of the method
    # (4 (N'+1) + 4 nnz + 3 N'/8 bytes per product, v and u bit-packed) per launch;
    # layout_*: the bytes of the compressed layout the kernel actually reads
    Bc = csr_step_bytes(info) * (products if sched.driver == lp.LP_DRIVER_PERSISTENT else 1)
    achieved = Bc / (kern_ms / 1e3) / 1e9
    layout_gbs = Bl / (kern_ms / 1e3) / 1e9
    copy_gbs = copy_probe(torch, dev, stream)
    log(f"[bench] {kname}: {kern_ms * 1e3:.2f} us/launch, {Bc / 1e6:.1f} MB algorithmic -> {achieved:.0f} GB/s; "
        f"layout {Bl / 1e6:.1f} MB -> {layout_gbs:.0f} GB/s (device copy probe: {copy_gbs:.0f} GB/s)")
    traffic = recorded_traffic(kname, B) if sched.driver != lp.LP_DRIVER_PERSISTENT else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname, "bytes_per_launch": Bc, "bytes": "algorithmic: int32 CSR step, "
                "4 (N'+1) + 4 nnz + 3 N'/8 bytes per product",
                "us_per_launch": round(kern_ms * 1e3, 3),
                "traffic_over_bytes": round(traffic / Bc, 4) if traffic else None,
                "copy_probe_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "layout": {"bytes_per_launch": Bl, "GB/s": round(layout_gbs, 1),
                           "frac": round(layout_gbs / HBM_PEAK_GBS, 4),
                           "traffic_over_bytes": round(traffic / Bl, 4) if traffic else None}}

    # serving first among the other legs, so that no state they leave behind (cached device
    # memory, schedules, transposes) weighs on its latencies
    serving = None if args.no_serving else bench_serving(args, gen, lp)

    # the frontier driver on the same matrix: end-to-end solve time (it visits each entry once per
    # solve, so its bytes are not those of the full-sweep product and no GB/s is claimed for it)
    frontier = None
    if not args.no_frontier:
        fs = lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER)
        t = time.perf_counter()
        fmodel, fprods = m.least_model(sched=fs, stream=stream)
        first_ms = (time.perf_counter() - t) * 1e3
        assert fprods == products and np.array_equal(fmodel, model), "frontier result differs from the full sweep"
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(args.steps):
            m.least_model(sched=fs, stream=stream)
        f1.record(stream)
        torch.cuda.synchronize()
        fms = f0.elapsed_time(f1) / max(args.steps, 1)
        frontier = {"driver": "frontier (semi-naive push through the transposed matrix)",
                    "ms_per_solve": round(fms, 4), "products": fprods,
                    "speedup_vs_full_sweep": round(ms_per_step / fms, 2),
                    "first_call_ms_with_transpose_build": round(first_ms, 1)}
        log(f"[bench] frontier: {frontier}")

    stable = None
    if not args.no_stable:
        q = gen.normal_uniform(args.seed)
        with lp.Matrix(q, stream=stream) as mq:
            mq.stable_models(stream=stream)
            torch.cuda.synchronize()
            reps = 20
            s0 = torch.cuda.Event(enable_timing=True)
            s1 = torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            for _ in range(reps):
                r = mq.stable_models(stream=stream)
            s1.record(stream)
            torch.cuda.synchronize()
            sms = s0.elapsed_time(s1) / reps
            H = 1 << mq.info["n_neg"]
            stable = {"workload": "normal_uniform: 10,000 atoms, 20,000 rules, bodies 1-5, 16 negated atoms",
                      "guesses": H, "ms_per_solve": round(sms, 3), "guesses_per_s": round(H / (sms / 1e3), 1),
                      "n_models": r["n_models"], "products": r["products"]}
            if not args.no_cpu_baseline:
                # the oracle's per-guess least models and Algorithm 3 test: one thread on guesses
                # 0..8191, and all 65,536 guesses over the host's threads (OpenMP)
                import oracle

                t = time.perf_counter()
                oracle.stable(q, guess_begin=0, guess_count=8192, threads=1)
                one = time.perf_counter() - t
                thr = cpu_threads()
                t = time.perf_counter()
                ro = oracle.stable(q, threads=thr)
                alls = time.perf_counter() - t
                assert np.array_equal(np.nonzero(ro["accept"])[0], lp.accepted_indices(r["accepted"])), \
                    "stable models differ from the oracle"
                stable["cpu_baseline"] = {"kind": "oracle", "unit": "guesses/s",
                                          "one_thread": {"value": round(8192 / one, 1), "cores": 1,
                                                         "sample": "guesses 0-8191"},
                                          "all_cores": {"value": round(H / alls, 1), "cores": thr,
                                                        "sample": "all 65,536 guesses"}}
        log(f"[bench] stable: {stable}")
        # guess sampling with local search where 2^K cannot be enumerated: a normal program with
        # 40 negated atoms (65,536 guesses per round, 4 rounds; every found model is sound)
        qs = gen.normal_uniform(args.seed, 10_000, 20_000, k_neg=40, p_neg=0.1)
        with lp.Matrix(qs, stream=stream) as ms:
            ms.stable_search(n_samples=1024, rounds=1, seed=1, stream=stream)
            t = time.perf_counter()
            sr = ms.stable_search(n_samples=65536, rounds=4, seed=2, max_found=4096, stream=stream)
            sdt = time.perf_counter() - t
            stable["search"] = {"workload": "normal_uniform: 10,000 atoms, 20,000 rules, 40 negated atoms "
                                            "(2^40 guesses)", "guesses": 4 * 65536, "rounds": 4,
                                "ms": round(sdt * 1e3, 3), "guesses_per_s": round(4 * 65536 / sdt, 1),
                                "models_found": sr["n_found"]}
        log(f"[bench] stable search: {stable['search']}")

    batch = None if args.no_batch else bench_batch(args, torch, gen, lp, stream)
    dense = None if args.no_dense else bench_dense(gen, lp, stream)
    small = bench_small(gen, lp, stream)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        times = []
        t_all = time.perf_counter()
        while True:
            t = time.perf_counter()
            omodel, oprods, _, _ = oracle.sd_fixpoint(prog)
            times.append(time.perf_counter() - t)
            if time.perf_counter() - t_all > args.cpu_budget_s or len(times) >= 10:
                break
        assert oprods == products and np.array_equal(omodel, model), "GPU result differs from the oracle"
        tmean = sum(times) / len(times)
        cpu = {"value": round(entries / tmean, 1), "unit": "entries/s", "cores": 1, "kind": "oracle",
               "sample": f"whole workload, {len(times)} solves of the oracle's standardized forward "
                         f"chaining (single thread, {tmean:.2f} s each, index build included)"}
        log(f"[bench] cpu oracle: {tmean:.3f} s/solve")

    out = {
        "metric": "rule-body entries/s per T_P step (GB/s vs HBM peak); stable-model guesses/s",
        "value": round(value, 1),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"chain_zipf: definite program, {n_atoms:,} atoms, "
                               f"{n_rules:,} rules, bodies 1-8, "
                               "1% facts, Zipf(1.1) heads, 2,000-long chain; least model, full-sweep products",
                   "seed": args.seed, "n_rows": info["n_rows"], "nnz": info["nnz"], "products": products,
                   "build_s": round(build_s, 3), "us_per_product": round(ms_per_step * 1e3 / products, 3),
                   "ms_per_step_p50": round(float(np.median(per_solve)), 4) if per_solve else None,
                   "ms_per_step_min": round(min(per_solve), 4) if per_solve else None},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "stable_models": stable,
        "batch": batch,
        "frontier": frontier,
        "dense": dense,
        "small_program": small,
        "serving": serving,
        "schedule": lp.schedule_dict(sched),
        "step_us_per_shape": variants or None,
    }
    print(json.dumps(out), flush=True)
    m.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
