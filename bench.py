#!/usr/bin/env python3
"""SOS solves/sec at 1e-4 residual on one MI355X.

A step is one batched solve of the whole workload from the cold start (or from the
learned warm start where the workload has one): every problem of the batch is run
to max(r_p, r_d, r_g) <= 1e-4 (FP64-measured) or to an infeasibility certificate.
Inputs are set up and resident in HBM before the timed region.

Prints ONE JSON line (see the README of the repository for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SOS solves/sec at 1e-4 residual: batched FP32+warm-start vs plain FP64 ADMM"
PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector peak
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------- workloads
def workload_pop_batch(count: int):
    from sosgen import families as F
    return [F.pop_batch_member(s) for s in range(count)]


def workload_lyapunov_test(count: int):
    from sosgen import families as F
    return [F.lyapunov(s) for s in range(3584, 3584 + count)]


WORKLOADS = {
    "pop_batch_512": dict(make=lambda: workload_pop_batch(512), count=512, plain_sample=4,
                          desc="512 unconstrained quartic POPs, n ~ U{6..16} (Gram 28..153, m 210..4845), "
                               "seeds 0..511, variables scaled, batched FP32 bulk + FP64 polish, cold start"),
    "lyapunov_512": dict(make=lambda: workload_lyapunov_test(512), count=512, plain_sample=32,
                         desc="512 Lyapunov programs, n = 6, quartic V (t = 203 free, Gram 28 and 84, m = 1134), "
                              "seeds 3584..4095, batched FP32 bulk + FP64 polish, cold start"),
}


def eig_flops(N: int) -> float:
    """Algorithmic flops of one PSD projection of an N x N block: 9 N^3 for a symmetric
    eigendecomposition with vectors (textbook count) + N^3 for the rebuild V max(L,0) V^T
    at half the eigenvalues positive (2 N^2 r with r = N/2)."""
    return 10.0 * N ** 3


def iter_flops(prob) -> float:
    """Algorithmic flops of one ADMM iteration: the PSD projections plus the affine step
    (two sparse products with A: 4 nnz, the Woodbury correction 4 nnz(A_f) + 2 k^2, and
    about 12 vector flops per entry of u)."""
    nnz = prob.A.nnz
    return sum(eig_flops(N) for N in prob.psd_dims) + 4.0 * nnz + 12.0 * (prob.n + prob.m)


# ----------------------------------------------------------------------------- CPU baseline
def cpu_baseline(probs, budget_s: float, tol: float):
    from threadpoolctl import threadpool_limits

    from oracle.admm import Oracle
    t0 = time.perf_counter()
    done, solved, names = 0, 0, []
    with threadpool_limits(limits=1):
        for p in probs:
            r = Oracle.from_problem(p).solve(tol=tol, max_iters=2000, check_every=10)
            done += 1
            solved += r.status in (1, 2, 3)
            names.append(f"seed{p.meta.get('seed')}(N={max(p.psd_dims)})")
            if time.perf_counter() - t0 > budget_s:
                break
    el = time.perf_counter() - t0
    return {"value": solved / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} problems of the workload solved one at a time in FP64 with I + A A^T "
                      f"factored directly, 1 BLAS thread: {', '.join(names)}; {el:.1f} s"}


# ----------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lyapunov_512", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--schedule", default=None, help="schedule JSON string or file")
    ap.add_argument("--plain-sample", type=int, default=0, help="0 = the workload's default")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; a batch would be split across GPUs by "
                                   "problem (see the design notes), which is not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1708_04174_amd import binding as B

    wl = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    probs = wl["make"]()
    log(f"[bench] generated {len(probs)} problems in {time.perf_counter() - t0:.1f}s")
    sched = args.schedule
    if sched and os.path.exists(sched):
        sched = open(sched).read()
    if sched is None:
        default_sched = os.path.join(ROOT, "paper_1708_04174_amd", "schedules", f"{args.workload}.json")
        if os.path.exists(default_sched):
            sched = open(default_sched).read()

    st = B.sos_default_settings(tol=args.tol, max_iters=2000, check_every=10,
                                precision=B.SOS_FP32_MIXED, polish_iters=1)
    t0 = time.perf_counter()
    works = [B.setup_problem(p, st) for p in probs]
    batch = B.sos_batch_setup(works, sched)
    log(f"[bench] setup {time.perf_counter() - t0:.1f}s")

    def one_step():
        B.sos_batch_reset(batch)
        torch.cuda.synchronize()
        infos = B.sos_batch_solve(batch)
        return infos, B.sos_batch_last_ms(batch), B.sos_batch_phase_ms(batch, 0), B.sos_batch_phase_ms(batch, 1)

    for i in range(args.warmup):
        infos, ms, p0, p1 = one_step()
        log(f"[bench] warmup {i}: {ms:.1f} ms (solve kernel {p0:.1f} ms, polish {p1:.1f} ms)")

    step_ms, k0_ms, k1_ms, counted = [], [], [], []
    fp32_iters = None
    for i in range(args.steps):
        torch.cuda.synchronize()
        infos, ms, p0, p1 = one_step()
        torch.cuda.synchronize()
        ok = [inf["status"] in (1, 2, 3) for inf in infos]
        step_ms.append(ms)
        k0_ms.append(p0)
        k1_ms.append(p1)
        counted.append(sum(ok))
        fp32_iters = [inf["iters"] - inf["polish_iters"] for inf in infos]
        log(f"[bench] step {i}: {ms:.1f} ms, {sum(ok)}/{len(ok)} solved "
            f"(solve kernel {p0:.1f} ms, polish {p1:.1f} ms)")

    total_ms = float(np.sum(step_ms))
    value = float(np.sum(counted)) / (total_ms / 1e3)
    statuses = {}
    for inf in infos:
        statuses[inf["status_name"]] = statuses.get(inf["status_name"], 0) + 1
    iters = np.array([inf["iters"] for inf in infos])
    worst = max(max(inf["res_pri"], inf["res_dual"], inf["gap"]) for inf in infos if inf["status"] == 1) \
        if any(inf["status"] == 1 for inf in infos) else None

    # roofline of the dominant kernel: the persistent FP32 solve kernel
    flops = sum(it * iter_flops(p) for it, p in zip(fp32_iters, probs))
    k_ms = float(np.mean(k0_ms))
    achieved = flops / (k_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                "kernel": "admm_persistent<float>", "kernel_ms": k_ms,
                "algorithmic_flops_per_launch": flops}

    # plain FP64 arm: one problem at a time, every step in FP64, cold start
    plain = None
    if not args.no_plain:
        ns = args.plain_sample or wl["plain_sample"]
        idx = np.linspace(0, len(probs) - 1, ns).astype(int)
        s64 = B.sos_default_settings(tol=args.tol, max_iters=2000, check_every=10, precision=B.SOS_FP64)
        tms, ok64 = 0.0, 0
        for i in idx:
            w = B.setup_problem(probs[i], s64)
            inf = B.sos_solve(w)
            tms += inf["solve_ms"]
            ok64 += inf["status"] in (1, 2, 3)
            w.free()
        plain = {"value": ok64 / (tms / 1e3), "unit": "solves/s", "sample": f"{len(idx)} problems spread over the "
                 "workload, sos_solve one at a time in FP64", "ms_total": tms}
        log(f"[bench] plain FP64: {plain['value']:.2f} solves/s")

    cpu = None
    if not args.no_cpu_baseline:
        order = sorted(range(len(probs)), key=lambda i: max(probs[i].psd_dims))
        sample = [probs[i] for i in order[::max(1, len(order) // 12)]]
        cpu = cpu_baseline(sample, args.cpu_budget, args.tol)
        log(f"[bench] cpu baseline: {cpu['value']:.3f} solves/s")

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "description": wl["desc"], "problems": len(probs),
                   "tol": args.tol, "statuses": statuses, "iters_median": float(np.median(iters)),
                   "iters_max": int(iters.max()), "worst_solved_residual": worst,
                   "phase_ms": {"solve_kernel": k_ms, "polish_kernel": float(np.mean(k1_ms))}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": (value / plain["value"]) if plain else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
