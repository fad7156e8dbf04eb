"""Times the batched least-model launch (many definite programs, Algorithm 1
per program, one launch) on one GPU and prints one JSON line.

The workload is the 512-program batch: atoms log-uniform in 1e3..1e5, rules
2x atoms, bodies 1..6, 2% facts. The plan's shape is autotuned first; then
--reps replays of its graph are timed with HIP events, and the results are
checked against single-program solves. With --copy-mb, one device-to-device
copy of that many MiB follows (a known-size kernel that calibrates byte
counters in a profile of the same run).

    python -m paper_2009_10247_amd.batch_solve [--reps 20] [--count 512] [--seed 0] [--shape 4,16,1024]
        [--frontier]

--shape wpw,unroll,block fixes the kernel shape instead of autotuning it (the
queue order and teams are still laid out by the product counts of a first
run, lp_batch_tune with reps 0), and --no-check skips the comparison with
single-program solves, so that a profile holds batch launches of one shape
only. --frontier times a frontier plan instead (the same programs solved by
frontier levels, each program's transposed matrix read once per solve).
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=0)
    ap.add_argument("--shape", default=None, help="wpw,unroll,block (no autotuning)")
    ap.add_argument("--no-check", action="store_true", help="skip the single-program solves (profiles)")
    ap.add_argument("--frontier", action="store_true", help="a frontier plan instead of matrix products")
    args = ap.parse_args(argv)
    import torch

    from . import gen, lp

    torch.cuda.init()
    st = torch.cuda.current_stream()
    progs = gen.batch_programs(args.seed, args.count)
    mats = [lp.Matrix(p, stream=st) for p in progs]
    try:
        sched = None
        if args.frontier:
            sched = lp.make_schedule(driver=lp.LP_DRIVER_FRONTIER)
        elif args.shape:
            sched = lp.lp_schedule()
            sched.wpw, sched.unroll, sched.block = (int(x) for x in args.shape.split(","))
        with lp.Batch(mats, sched=sched, stream=st) as plan:
            if args.frontier:
                pass
            elif args.shape:
                plan.tune(reps=0, stream=st)  # order and teams by product counts, at the given shape
            elif not args.no_tune:
                plan.tune(reps=3, stream=st)
            plan.run(stream=st)
            res = plan.results(stream=st)
            for m, (g, pr) in ([] if args.no_check else zip(mats, res)):
                g2, pr2 = m.least_model(stream=st)
                assert pr == pr2 and (g == g2).all(), "batch result differs from the single-program solve"
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(args.reps):
                plan.run(stream=st)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / max(args.reps, 1)
            info = plan.info()
            prods = [pr for _, pr in res]
            entries = sum(m.info["nnz"] * pr for m, pr in zip(mats, prods))
            # int32-CSR bytes of every product: 4 (N'+1) + 4 nnz + 3 N'/8 per product
            csr = sum((4 * (m.info["n_rows"] + 1) + 4 * m.info["nnz"] + 3 * ((m.info["n_rows"] + 7) // 8)) * pr
                      for m, pr in zip(mats, prods))
            print(json.dumps({"workload": f"{args.count} definite programs, atoms log-uniform 1e3-1e5, rules 2x "
                                          "atoms, bodies 1-6, 2% facts; one batch launch (graph replay)",
                              "ms_per_batch": round(ms, 4),
                              "entries_per_s": None if args.frontier else round(entries / (ms / 1e3), 1),
                              "products_total": int(sum(prods)), "nnz": info["nnz"],
                              # (a frontier plan does not read the matrix once per product: no CSR rate for it)
                              "csr_bytes_per_batch": int(csr),
                              "csr_GB/s": None if args.frontier else round(csr / (ms / 1e3) / 1e9, 1),
                              "plan": "frontier" if args.frontier else "matrix products",
                              # the transposed matrices, which a frontier plan reads once per solve
                              "transpose_bytes": int(sum(4 * (m.info["n_rows"] + 1) + 4 * m.info["nnz"]
                                                         for m in mats)),
                              "shape": {k: info[k] for k in ("wpw", "unroll", "block", "grid", "lds_bytes")},
                              "teams": {k: info[k] for k in ("n_teams", "team_members", "team_fallbacks")}}),
                  flush=True)
        if args.copy_mb:
            n = args.copy_mb << 20
            src = torch.ones(n // 4, dtype=torch.int32, device="cuda")
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
    finally:
        for m in mats:
            m.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
