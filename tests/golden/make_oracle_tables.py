#!/usr/bin/env python3
"""Writes tests/golden/oracle_tables.json: results of the FP64 CPU oracle (oracle/admm.py) on
full-size seeded workloads that are too slow to re-solve inside a GPU test or the benchmark.

This script calls only the input generators (sosgen/) and the oracle; no value in the table
comes from the GPU library.  Entries:

* lyapunov_512: status and iterations of the 512 held-out Lyapunov programs (seeds
  3584..4095; n = 6, quartic V, Gram blocks 28 and 84), tol 1e-4, 2000 iterations, residual
  checks every 10 iterations, cold start: the settings the benchmark solves them with.  The
  benchmark counts a GPU result only where its status equals the oracle's.
* ball_pop_n16: gamma of the constrained quartic POP on the unit ball, n = 16 (Gram blocks
  153 and 17, m = 4845), seeds 0..2, solved to tol 1e-7 (the reference for the mixed-precision
  gamma error), and the status at tol 1e-4 / 2000 iterations.
* pop_n20: status and iterations of the unconstrained quartic POP n = 20 with N(0, 0.1) quartic
  cross terms (Gram block 231, m = 10626), seed 0, tol 1e-4, 2000 iterations.
* example_pop_n24: the test POP of Section VII-A at n = 24 (blocks 325 and 25, m = 20475; Table
  I's n = 24 row), status, iterations and gamma at tol 1e-4 / 2000 iterations, and gamma at tol 1e-7
  (compared with the brute-force minimum by a CPU test).

Usage: python tests/golden/make_oracle_tables.py [--only KEY ...] [--workers N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "oracle_tables.json")


def _solve(args):
    kind, seed, tol, max_iters = args
    from threadpoolctl import threadpool_limits

    from oracle.admm import Oracle
    from sosgen import families as F
    make = {"lyapunov": F.lyapunov, "ball16": lambda s: F.pop_ball(16, s),
            "pop20": lambda s: F.pop_unconstrained(20, s, cross_std=0.1),
            "example": lambda s: F.example_pop(s)}[kind]
    t = time.perf_counter()
    with threadpool_limits(limits=1):
        r = Oracle.from_problem(make(seed)).solve(tol=tol, max_iters=max_iters, check_every=10)
    out = {"status": int(r.status), "iters": int(r.iters), "seconds": round(time.perf_counter() - t, 2)}
    if r.status == 1 and kind != "lyapunov":     # Lyapunov programs have no gamma (c = 0)
        out["gamma"] = float(r.x[0])
        out["residual"] = float(max(r.res_pri, r.res_dual, r.gap))
    return kind, seed, tol, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    table = json.load(open(OUT)) if os.path.exists(OUT) else {}
    jobs = []
    want = set(args.only) if args.only else {"lyapunov_512", "ball_pop_n16", "pop_n20", "example_pop_n24"}
    if "lyapunov_512" in want:
        jobs += [("lyapunov", s, 1e-4, 2000) for s in range(3584, 4096)]
    if "ball_pop_n16" in want:
        jobs += [("ball16", s, 1e-7, 50000) for s in range(3)] + [("ball16", s, 1e-4, 2000) for s in range(3)]
    if "pop_n20" in want:
        jobs += [("pop20", 0, 1e-4, 2000)]
    if "example_pop_n24" in want:
        jobs += [("example", 24, 1e-4, 2000), ("example", 24, 1e-7, 20000)]
    # slowest first, so the pool's tail is short
    jobs.sort(key=lambda j: {"example": 0, "ball16": 0, "pop20": 1, "lyapunov": 2}[j[0]])
    res = {}
    with ProcessPoolExecutor(max_workers=args.workers) as ex:
        for kind, seed, tol, out in ex.map(_solve, jobs):
            res[(kind, seed, tol)] = out
            print(kind, seed, tol, out, flush=True)
    common = {"oracle": "oracle/admm.py, FP64, I + A A^T factored directly, cold start u = v = (0, 0, 1), "
                        "alpha 1, residual checks every 10 iterations",
              "written_by": "tests/golden/make_oracle_tables.py"}
    if "lyapunov_512" in want:
        table["lyapunov_512"] = dict(common, tol=1e-4, max_iters=2000,
                                     seeds={str(s): res[("lyapunov", s, 1e-4)] for s in range(3584, 4096)})
    if "ball_pop_n16" in want:
        table["ball_pop_n16"] = dict(common, gamma_tol=1e-7, gamma_max_iters=50000,
                                     seeds={str(s): {"reference": res[("ball16", s, 1e-7)],
                                                     "tol_1e-4": res[("ball16", s, 1e-4)]} for s in range(3)})
    if "pop_n20" in want:
        table["pop_n20"] = dict(common, tol=1e-4, max_iters=2000, cross_std=0.1,
                                seeds={"0": res[("pop20", 0, 1e-4)]})
    if "example_pop_n24" in want:
        table["example_pop_n24"] = dict(common, n=24, tol=1e-4, max_iters=2000, result=res[("example", 24, 1e-4)],
                                        tight=dict(tol=1e-7, max_iters=20000, result=res[("example", 24, 1e-7)]))
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
