"""Times stable-model solves (Algorithms 2 and 3) of the normal program with
10,000 atoms, 20,000 rules and 16 negated atoms (65,536 guesses) on one GPU,
with the default products by dirty rows or, with --full-sweep, products that
evaluate every row. Prints one JSON line.

    python -m paper_2009_10247_amd.stable_solve [--reps 10] [--full-sweep]
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--full-sweep", action="store_true")
    args = ap.parse_args(argv)
    import torch

    from . import gen, lp

    torch.cuda.init()
    st = torch.cuda.current_stream()
    p = gen.normal_uniform(args.seed)
    flags = lp.LP_STABLE_FULL_SWEEP if args.full_sweep else 0
    with lp.Matrix(p, flags=flags, stream=st) as m:
        r = m.stable_models(stream=st)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.reps):
            r = m.stable_models(stream=st)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(args.reps, 1)
        H = 1 << m.info["n_neg"]
        print(json.dumps({"workload": "normal_uniform: 10,000 atoms, 20,000 rules, 16 negated atoms",
                          "driver": "full sweep" if args.full_sweep else "dirty rows", "guesses": H,
                          "ms_per_solve": round(ms, 4), "guesses_per_s": round(H / (ms / 1e3), 1),
                          "products": r["products"], "n_models": r["n_models"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
