"""Times least-model solves (Algorithm 1) on one GPU and prints one JSON line.

Programs (--program):
  chain  the definite program with 1,000,000 atoms, 5,000,000 rules and a
         2,000-long derivation chain; --driver frontier (default: semi-naive
         pushes through the transposed matrix) or batched (full-sweep products);
  small  the 1,000-atom definite program (2,000 rules, 5% facts, bodies 1-4)
         with the default driver, which runs the whole loop in one workgroup;
         wall-clock time per solve, model in host memory.

    python -m paper_2009_10247_amd.least_solve [--reps 10] [--program chain|small] [--driver frontier|batched]
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--program", choices=("chain", "small"), default="chain")
    ap.add_argument("--driver", choices=("frontier", "batched"), default="frontier")
    args = ap.parse_args(argv)
    import torch

    from . import gen, lp

    torch.cuda.init()
    st = torch.cuda.current_stream()
    if args.program == "small":
        p = gen.definite_uniform(args.seed, 1000, 2000, 0.05, 4)
        with lp.Matrix(p, stream=st) as m:
            m.least_model(stream=st)
            t = time.perf_counter()
            for _ in range(args.reps):
                model, prods = m.least_model(stream=st)
            us = (time.perf_counter() - t) * 1e6 / max(args.reps, 1)
            print(json.dumps({"workload": "definite_uniform: 1,000 atoms, 2,000 rules, 5% facts, bodies 1-4",
                              "driver": "default", "us_per_solve": round(us, 1), "products": prods,
                              "n_rows": m.info["n_rows"], "model_size": int(model.sum())}), flush=True)
        return 0
    p = gen.chain_zipf(args.seed)
    drv = lp.LP_DRIVER_FRONTIER if args.driver == "frontier" else lp.LP_DRIVER_BATCHED
    sched = lp.make_schedule(driver=drv)
    with lp.Matrix(p, stream=st) as m:
        _, prods = m.least_model(sched=sched, stream=st)  # the frontier driver builds its transpose here
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.reps):
            model, prods = m.least_model(sched=sched, stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(args.reps, 1)
        print(json.dumps({"workload": "chain_zipf: 1,000,000 atoms, 5,000,000 rules, 2,000-long chain",
                          "driver": args.driver, "ms_per_solve": round(ms, 4), "products": prods,
                          "model_size": int(model.sum())}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
