"""Times least-model solves (Algorithm 1) of the definite program with
1,000,000 atoms, 5,000,000 rules and a 2,000-long derivation chain on one GPU,
with the frontier driver (semi-naive pushes through the transposed matrix) or,
with --driver batched, full-sweep products. Prints one JSON line.

    python -m paper_2009_10247_amd.least_solve [--reps 10] [--driver frontier|batched]
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--driver", choices=("frontier", "batched"), default="frontier")
    args = ap.parse_args(argv)
    import torch

    from . import gen, lp

    torch.cuda.init()
    st = torch.cuda.current_stream()
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
