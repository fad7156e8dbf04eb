"""Serving driver: Poisson arrivals of least-model and stable-model queries
against the native request loop (lp_server_*), with latency percentiles and
throughput per arrival rate.

Requests draw their program from a pool with Zipf(1.0) popularity; a program
without negation is a least-model query, one with K > 0 negated atoms a
stable-model query. Before the timed streams every pool program is solved
once alone on an idle server; every result of the streams is then compared
byte for byte with that alone result.

    python -m paper_2009_10247_amd.serve [--rates 10,30,100,300,1000]
        [--requests 2000] [--pool 256] [--hi 1e6] [--slots 4]
"""
from __future__ import annotations

import argparse
import json
import sys
import threading
import time

import numpy as np

from . import gen, lp


def zipf_weights(n: int, s: float = 1.0) -> np.ndarray:
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    return w / w.sum()


def _collect(server, n, out, deadline, progress=None):
    got = 0
    t_log = time.perf_counter()
    while got < n and time.perf_counter() < deadline:
        info = server.wait_any(500)
        if progress is not None and time.perf_counter() - t_log > 30.0:
            t_log = time.perf_counter()
            progress(f"{got}/{n} requests completed")
        if info is None:
            continue
        model, acc = server.take_result(info["request_id"], info["program_id"])
        out[info["request_id"]] = (info, model, acc)
        got += 1


def solve_alone(server, pids, timeout_s: float = 600.0) -> dict:
    """Each program solved by itself on the (idle) server: pid -> (model, accepted, products)."""
    ref = {}
    for pid in pids:
        rid = server.submit(pid)
        t_end = time.perf_counter() + timeout_s
        info = None
        while info is None and time.perf_counter() < t_end:
            info = server.wait_any(1000)
        if info is None or info["request_id"] != rid:
            raise RuntimeError(f"alone solve of program {pid} did not complete")
        if info["status"] != 0:
            raise lp.LPError(info["status"], f"program {pid}")
        model, acc = server.take_result(rid, pid)
        ref[pid] = (model, acc, info["products"], info["n_models"])
    return ref


def run_stream(server, pids, weights, rate: float, n_requests: int, seed: int, ref: dict | None = None,
               timeout_s: float = 900.0, progress=None) -> dict:
    """Submit n_requests at Poisson(rate) arrival times; return latency and
    throughput statistics. With ref, every result is compared with it.
    progress (nullable) receives a status line about every 30 s."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    choice = rng.choice(len(pids), size=n_requests, p=weights)
    results = {}
    collector = threading.Thread(target=_collect,
                                 args=(server, n_requests, results, time.perf_counter() + timeout_s, progress))
    collector.start()
    t0 = time.perf_counter()
    late = 0.0
    for i in range(n_requests):
        dt = t0 + arrivals[i] - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        else:
            late = max(late, -dt)
        server.submit(pids[choice[i]])
    collector.join()
    if len(results) != n_requests:
        raise RuntimeError(f"{n_requests - len(results)} requests did not complete")
    infos = [r[0] for r in results.values()]
    bad = [i for i in infos if i["status"] != 0]
    if bad:
        raise lp.LPError(bad[0]["status"], f"request {bad[0]['request_id']}")
    mismatches = 0
    if ref is not None:
        for info, model, acc in results.values():
            m0, a0, p0, n0 = ref[info["program_id"]]
            same = (np.array_equal(model, m0) and info["products"] == p0 and info["n_models"] == n0 and
                    (a0 is None or np.array_equal(acc, a0)))
            mismatches += 0 if same else 1
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos]) * 1e3
    wait = np.array([i["t_start"] - i["t_submit"] for i in infos]) * 1e3
    t_first = min(i["t_submit"] for i in infos)
    t_last = max(i["t_done"] for i in infos)
    span = max(t_last - t_first, 1e-9)
    entries = sum(i["nnz"] * i["products"] for i in infos)
    kinds = np.array([i["kind"] for i in infos])
    return {
        "rate": rate, "requests": n_requests,
        "least": int((kinds == 0).sum()), "stable": int((kinds == 1).sum()),
        "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
        "p50_least_ms": round(float(np.percentile(lat[kinds == 0], 50)), 3) if (kinds == 0).any() else None,
        "p50_stable_ms": round(float(np.percentile(lat[kinds == 1], 50)), 3) if (kinds == 1).any() else None,
        "p99_queue_ms": round(float(np.percentile(wait, 99)), 3),
        "completed_per_s": round(n_requests / span, 1), "entries_per_s": round(entries / span, 1),
        "batched": int(sum(1 for i in infos if i["batch_size"] > 1)),
        "batched_stable": int(sum(1 for i in infos if i["batch_size"] > 1 and i["kind"] == 1)),
        "mean_batch": round(float(np.mean([i["batch_size"] for i in infos])), 2),
        "uploads": int(sum(i["built"] for i in infos)),
        "submit_late_max_ms": round(late * 1e3, 3),
        "mismatches": mismatches if ref is not None else None,
    }


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="10,30,100,300,1000")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--lo", type=float, default=1e3)
    ap.add_argument("--hi", type=float, default=1e6)
    ap.add_argument("--max-k", type=int, default=12)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--batch-max", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gb", type=float, default=0.0)
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    t = time.perf_counter()
    t_log = [t]

    def every_30s(msg):
        if time.perf_counter() - t_log[0] > 30.0:
            t_log[0] = time.perf_counter()
            log(f"[serve] {msg}")

    pool = gen.serving_pool(args.seed, args.pool, args.lo, args.hi, max_k=args.max_k,
                            progress=lambda i: every_30s(f"{i}/{args.pool} programs drawn"))
    log(f"[serve] pool of {len(pool)} programs generated in {time.perf_counter() - t:.1f}s")
    with lp.Server(n_slots=args.slots, batch_max=args.batch_max,
                   hbm_budget=int(args.budget_gb * 2**30)) as srv:
        t = time.perf_counter()
        pids = []
        for p in pool:
            pids.append(srv.add_program(p))
            every_30s(f"{len(pids)}/{len(pool)} programs registered")
        log(f"[serve] registered in {time.perf_counter() - t:.1f}s")
        t = time.perf_counter()
        ref = solve_alone(srv, pids)
        log(f"[serve] alone solves (uploads included) in {time.perf_counter() - t:.1f}s")
        weights = zipf_weights(len(pids))
        rows = []
        for k, rate in enumerate(float(x) for x in args.rates.split(",")):
            row = run_stream(srv, pids, weights, rate, args.requests, args.seed + 1 + k, ref,
                             progress=lambda msg, r=rate: log(f"[serve] rate {r:g}: {msg}"))
            log(f"[serve] {json.dumps(row)}")
            rows.append(row)
        st = srv.stats()
    out = {"workload": f"serving: pool of {args.pool} programs (atoms log-uniform {args.lo:g}-{args.hi:g}, "
                       f"rules 3x atoms, bodies 1-6, 2% facts, K ~ U{{0..{args.max_k}}}), Zipf(1.0) popularity, "
                       f"Poisson arrivals",
           "slots": args.slots, "rates": rows, "server": st}
    print(json.dumps(out), flush=True)
    return 0 if all(r["mismatches"] == 0 for r in rows) else 1


if __name__ == "__main__":
    sys.exit(main())
