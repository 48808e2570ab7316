"""Autotuner for the batched solver's launch schedule.

Times fixed-length batched runs (the same persistent kernel the solve uses, stopped after
a fixed number of iterations) and picks
  1. per block-size bucket (N < 32, 64, 96, 128, 192, 256, larger): the lanes that
     share one Jacobi column pair (8, 16 or 32) in the lane-group form of the
     eigensolver (blocks too large for the LDS form);
  2. for the whole batch: the eigensolver form for blocks that fit in LDS (rows split
     over the wavefronts for every block or from N = 128 on, or lane groups throughout),
     threads per workgroup and
     resident workgroups per CU (which also sets the LDS each workgroup may use).
Writes the schedule JSON that sos_batch_setup reads.

    python -m paper_1708_04174_amd.autotune --workload lyapunov --out schedules/lyapunov_512.json
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from collections import defaultdict

import numpy as np

from . import binding as B
from . import workloads as WL

BUCKETS = [32, 64, 96, 128, 192, 256, 1 << 30]
KEYS = ["gs_n32", "gs_n64", "gs_n96", "gs_n128", "gs_n192", "gs_n256", "gs_big"]


def bucket_of(N: int) -> int:
    for i, b in enumerate(BUCKETS):
        if N < b:
            return i
    return len(BUCKETS) - 1


def time_schedule(works, sched: dict, reps: int = 2) -> float:
    """Best-of-reps time of a fixed-length batched run: the FP32 run of `works` plus the FP64
    run of the same problems (the mixed form spends a hard problem's iterations in both)."""
    total = 0.0
    for ws in works:
        bt = B.sos_batch_setup(ws, json.dumps(sched))
        best = np.inf
        for _ in range(reps):
            B.sos_batch_reset(bt)
            B.sos_batch_solve(bt)
            best = min(best, B.sos_batch_phase_ms(bt, 0) + max(0.0, B.sos_batch_phase_ms(bt, 1)))
        bt.free()
        total += best
    return total


def _fixed_length_works(probs, iters: int):
    """(FP32-only, FP64) handles for fixed-length runs: an unreachable tolerance, and for the
    FP32 run no stall hand-over (the iteration budget is all FP32 but the last one)."""
    s32 = B.sos_default_settings(tol=1e-14, max_iters=iters, precision=B.SOS_FP32_MIXED, polish_iters=1)
    s64 = B.sos_default_settings(tol=1e-14, max_iters=iters, precision=B.SOS_FP64)
    return [B.setup_problem(p, s32) for p in probs], [B.setup_problem(p, s64) for p in probs]


def tune(probs, precision: int = 0, iters: int = 40, sample: int = 64, log=print) -> dict:
    """precision is kept for the call signature; every candidate is timed in both precisions."""
    # fixed-length runs: an unreachable tolerance makes every problem run `iters` iterations
    # lanes per pair are tuned with the lane-group form on every block (eig_wave 0), so that
    # each bucket's choice is timed where it applies
    base = {"block_threads": 512, "wg_per_cu": 1, "max_sweeps": 60, "warm_eig": 1, "use_graph": 0, "eig_wave": 0,
            "rows_nmin": 0}
    byb = defaultdict(list)
    for i, p in enumerate(probs):
        for b in sorted({bucket_of(N) for N in p.psd_dims if N > 1}):
            byb[b].append(i)
    sched = dict(base)
    for k in KEYS:
        sched[k] = 16
    for b, idx in sorted(byb.items()):
        sub = [probs[i] for i in idx[:sample]]
        works = _fixed_length_works(sub, iters)
        res = {}
        for gs in (8, 16, 32):
            s = dict(sched)
            s[KEYS[b]] = gs
            res[gs] = time_schedule(works, s)
        sched[KEYS[b]] = min(res, key=res.get)
        log(f"[tune] bucket N<{BUCKETS[b]}: {len(sub)} problems, ms by lanes/pair {res} -> {sched[KEYS[b]]}")
        for ws in works:
            for w in ws:
                w.free()
    rng = np.random.default_rng(0)
    pick = rng.choice(len(probs), size=min(len(probs), 4 * sample), replace=False)
    works = _fixed_length_works([probs[i] for i in pick], iters)
    res = {}
    # eigensolver forms: (eig_wave, rows_nmin) = rows form for every block that fits in LDS,
    # rows form from N = 128 on (lane groups below: the single-solve default), lane groups for
    # every block
    for ew, rmin in ((2, 0), (2, 128), (0, 0)):
        for thr in (256, 512):
            for wpc in (1, 2):
                s = dict(sched)
                s["eig_wave"], s["rows_nmin"], s["block_threads"], s["wg_per_cu"] = ew, rmin, thr, wpc
                key = (ew, rmin, thr, wpc)
                res[key] = time_schedule(works, s)
                log(f"[tune] eigensolver form {ew} rows from N={rmin} threads {thr} wg/CU {wpc}: "
                    f"{res[key]:.2f} ms")
    ew, rmin, thr, wpc = min(res, key=res.get)
    sched["eig_wave"], sched["rows_nmin"], sched["block_threads"], sched["wg_per_cu"] = ew, rmin, thr, wpc
    sched["use_graph"] = 1
    for ws in works:
        for w in ws:
            w.free()
    sched["tuned"] = {"iters": iters, "runs": "fixed-length FP32 and FP64 batches, times added",
                      "problems": len(probs), "when": time.strftime("%Y-%m-%d")}
    return sched


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["lyapunov", "pop_batch"], default="lyapunov")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--out", required=True)
    ap.add_argument("--iters", type=int, default=40)
    ap.add_argument("--sample", type=int, default=64)
    a = ap.parse_args()
    import torch
    assert torch.cuda.is_available()
    seeds = WL.LYAP_TEST if a.workload == "lyapunov" else range(a.count)
    probs = WL.generate(a.workload, list(seeds)[:a.count])
    prec = B.SOS_FP32_MIXED if a.precision == "fp32" else B.SOS_FP64
    sched = tune(probs, prec, iters=a.iters, sample=a.sample, log=lambda m: print(m, file=sys.stderr, flush=True))
    with open(a.out, "w") as f:
        json.dump(sched, f, indent=1)
    print(json.dumps(sched))


if __name__ == "__main__":
    main()
