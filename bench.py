#!/usr/bin/env python3
"""SOS solves/sec at 1e-4 residual on one MI355X.

A step is one pass of the whole path over one batch of synthetic SOS programs with
inputs already resident on the GPU: the learned warm start (MLP inference on the
device, the warm-start kernel), the batched persistent solve (FP32 bulk, FP64 Schur
solve / theta / tau-kappa / residuals, FP64 polish), and cold re-solves of whatever the
warm start left unsolved.  A solve counts when its FP64 max(r_p, r_d, r_g) <= 1e-4 or
it ends in an infeasibility certificate, and only where the FP64 CPU oracle reaches the
same status (a stored table written by tests/golden/make_oracle_tables.py, which calls only
the oracle and the input generators).

Default workload: 512 held-out Lyapunov programs (n = 6, quartic V; Gram blocks 28 and
84, m = 1134).  The warm-start model is trained beforehand (untimed) on the solver's
own cold solutions of the 3584 training programs of the same family.

Prints ONE JSON line.
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
OK_STATUS = (1, 2, 3)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def eig_flops(N: int) -> float:
    """Algorithmic flops of one PSD projection of an N x N block: 9 N^3 for a symmetric
    eigendecomposition with vectors (textbook count) + N^3 for the rebuild V max(L,0) V^T
    at half the eigenvalues positive (2 N^2 r with r = N/2)."""
    return 10.0 * N ** 3


def iter_flops(prob) -> float:
    """Algorithmic flops of one ADMM iteration: the PSD projections plus the affine step
    (two sparse products with A: 4 nnz; Woodbury correction about 4 nnz(A_f) + 2 k^2;
    about 12 flops per entry of u)."""
    k = prob.n_free
    return sum(eig_flops(N) for N in prob.psd_dims) + 4.0 * prob.A.nnz + 2.0 * k * k + 12.0 * (prob.n + prob.m)


def _oracle_job(job):
    """One oracle solve in a worker process (1 BLAS thread): (seed, status, setup_s, solve_s)."""
    kind, seed, tol = job
    from threadpoolctl import threadpool_limits

    from oracle.admm import Oracle
    from sosgen import families as F
    prob = F.lyapunov(seed) if kind == "lyapunov" else F.pop_batch_member(seed)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        o = Oracle.from_problem(prob)
        t1 = time.perf_counter()
        r = o.solve(tol=tol, max_iters=2000, check_every=10)
        t2 = time.perf_counter()
    return seed, int(r.status), t1 - t0, t2 - t1


def _warm_worker(_):
    import scipy.sparse  # noqa: F401  - imports paid before the timed window

    import oracle.admm  # noqa: F401
    import sosgen.families  # noqa: F401
    return os.getpid()


def host_cpu():
    """(logical CPUs, CPUs this process may run on, CPU model name) of the host."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return os.cpu_count() or 1, avail, model


def cpu_baseline(kind: str, seeds, budget_s: float, tol: float, ok_status):
    """The oracle over a process pool on the host cores (at most 16 workers, one BLAS thread
    each), fed the workload's problems in the given order until budget_s of wall time has
    passed.  Throughput counts solve time only (the oracle's set-up, factoring I + A A^T, is
    reported apart), like the GPU arm, whose set-up is also reported apart."""
    import multiprocessing as mp
    nproc, avail, model = host_cpu()
    workers = max(1, min(16, avail))
    for var in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"   # inherited by the spawned workers
    ctx = mp.get_context("spawn")   # fresh interpreters: nothing of this process's GPU state
    pool = ctx.Pool(workers)
    try:
        pool.map(_warm_worker, range(workers))
        t0 = time.perf_counter()
        done, counted, setup_s, solve_s, t_last = 0, 0, 0.0, 0.0, 0.0
        for seed, status, su, so in pool.imap_unordered(_oracle_job, [(kind, int(s), tol) for s in seeds]):
            done += 1
            counted += ok_status(seed, status)
            setup_s += su
            solve_s += so
            t_last = time.perf_counter() - t0
            if t_last > budget_s:
                break
    finally:
        pool.terminate()
        pool.join()
    return {"value": workers * counted / solve_s if solve_s > 0 else None, "unit": "solves/s", "cores": workers,
            "kind": "oracle",
            "value_with_setup": workers * counted / (setup_s + solve_s) if solve_s > 0 else None,
            "wall_value": counted / t_last if t_last > 0 else None,
            "setup_ms_per_problem": 1e3 * setup_s / max(done, 1),
            "nproc": nproc, "cpus_available": avail, "cpu_model": model,
            "sample": f"{done} problems of the workload in a seeded random order, solved by a pool of {workers} "
                      f"worker processes until {budget_s:.0f} s of wall time had passed (FP64, I + A A^T factored "
                      f"directly, 1 BLAS thread each); {counted} counted; value = workers x counted / summed "
                      f"solve time (set-up excluded, as in the GPU arm)"}


COPY_PROBE_BYTES = 256 * 1024 * 1024

PER_ITER_CASES = {
    # name: (generator, description)
    "lyapunov": (lambda F: F.lyapunov(3584), "Lyapunov program, seed 3584: blocks 84 + 28, m = 1134, k = 203"),
    "pop_n6": (lambda F: F.pop_unconstrained(6, 0), "quartic POP n = 6: block 28, m = 210"),
    "pop_n10": (lambda F: F.pop_unconstrained(10, 0), "quartic POP n = 10: block 66, m = 1001"),
    "pop_n14": (lambda F: F.pop_unconstrained(14, 0), "quartic POP n = 14: block 120, m = 3060"),
    "ball_n16": (lambda F: F.pop_ball(16, 0), "ball POP n = 16: blocks 153 + 17, m = 4845, k = 154"),
    "pop_n20": (lambda F: F.pop_unconstrained(20, 0, cross_std=0.1), "quartic POP n = 20: block 231, m = 10626"),
}


# Section VII-A, Table I: CDCS-sos CPU seconds (2.8 GHz Core i7, tol 1e-3, at most 2000
# iterations) for the test POP's order-2 ball relaxation, and its Table III objective values
TABLE1_CDCS_S = {10: 0.4, 12: 0.7, 14: 1.4, 17: 3.5, 20: 8.5, 24: 22.8, 29: 67.1, 35: 216.9, 42: 686.6}
TABLE3_CDCS_GAMMA = {10: -9.10, 12: -11.11, 14: -13.12, 17: -16.06, 20: -19.08, 24: -23.15, 29: -28.17,
                     35: -34.08, 42: -41.05}


def table1(ns, tol: float):
    """The paper's test POP (Section VII-A) at the sizes of Table I, solved in FP64 by sos_solve
    (the multi-workgroup form from N = 128) at the paper's tolerance; seconds from the solve's
    own device timing, set-up apart."""
    from paper_1708_04174_amd import binding as B
    from sosgen import families as F
    out = []
    for n in ns:
        t0 = time.perf_counter()
        prob = F.example_pop(n)
        gen_s = time.perf_counter() - t0
        w = B.setup_problem(prob, B.sos_default_settings(tol=tol, max_iters=2000))
        inf = B.sos_solve(w)
        x, _, _ = B.sos_get_solution(w) if inf["tau"] > 0 else (np.full(1, np.nan), None, None)
        w.free()
        rec = {"n": n, "N": max(prob.psd_dims), "m": prob.m, "status": inf["status_name"], "iters": inf["iters"],
               "gamma": float(x[0]), "solve_s": inf["solve_ms"] / 1e3, "setup_s": inf["setup_ms"] / 1e3,
               "ms_per_iter": inf["solve_ms"] / max(inf["iters"], 1), "sweeps": inf["eig_sweeps"],
               "affine_ms_per_iter": inf["affine_ms"] / max(inf["iters"], 1),
               "projection_ms_per_iter": inf["eig_ms"] / max(inf["iters"], 1), "residual_ms": inf["resid_ms"],
               "generate_s": gen_s, "paper_cdcs_s": TABLE1_CDCS_S.get(n), "paper_cdcs_gamma": TABLE3_CDCS_GAMMA.get(n)}
        log(f"[table1] n {n}: N {rec['N']}, m {rec['m']}: {rec['status']} in {rec['iters']} iterations, "
            f"gamma {rec['gamma']:.4f}, {rec['solve_s']:.2f} s ({rec['ms_per_iter']:.2f} ms/iter; paper's CDCS-sos "
            f"{rec['paper_cdcs_s']} s, gamma {rec['paper_cdcs_gamma']})")
        out.append(rec)
    return out


# Section VII-B, Table II: sizes (N, m, t) and CDCS-sos CPU seconds (same machine and settings as
# Table I) for the local Lyapunov programs of random cubic systems
TABLE2 = {10: (65, 1100, 110, 0.3), 12: (90, 1963, 156, 0.4), 14: (119, 3255, 210, 0.6), 17: (170, 6273, 306, 1.1),
          20: (230, 11025, 420, 2.4), 24: (324, 21050, 600, 5.1), 29: (464, 41760, 870, 14.3),
          35: (665, 83475, 1260, 37.4), 42: (945, 164948, 1806, 92.8)}


def table2(ns, tol: float, seed: int = 0):
    """Table II's programs (sosgen.families.lyapunov_local, one random system per n) solved in FP64
    by sos_solve at the paper's tolerance; seconds from the solve's device timing, set-up apart."""
    from paper_1708_04174_amd import binding as B
    from sosgen import families as F
    out = []
    for n in ns:
        t0 = time.perf_counter()
        prob = F.lyapunov_local(n, seed)
        gen_s = time.perf_counter() - t0
        w = B.setup_problem(prob, B.sos_default_settings(tol=tol, max_iters=2000))
        inf = B.sos_solve(w)
        w.free()
        paper = TABLE2.get(n)
        rec = {"n": n, "N": max(prob.psd_dims), "m": prob.m, "t": prob.n_free, "status": inf["status_name"],
               "iters": inf["iters"], "solve_s": inf["solve_ms"] / 1e3, "setup_s": inf["setup_ms"] / 1e3,
               "ms_per_iter": inf["solve_ms"] / max(inf["iters"], 1), "sweeps": inf["eig_sweeps"],
               "affine_ms_per_iter": inf["affine_ms"] / max(inf["iters"], 1),
               "projection_ms_per_iter": inf["eig_ms"] / max(inf["iters"], 1), "residual_ms": inf["resid_ms"],
               "generate_s": gen_s, "paper_N_m_t": paper[:3] if paper else None,
               "paper_cdcs_s": paper[3] if paper else None}
        log(f"[table2] n {n}: N {rec['N']}, m {rec['m']}, t {rec['t']}: {rec['status']} in {rec['iters']} "
            f"iterations, {rec['solve_s']:.2f} s ({rec['ms_per_iter']:.2f} ms/iter); paper's sizes "
            f"{rec['paper_N_m_t']}, CDCS-sos {rec['paper_cdcs_s']} s")
        out.append(rec)
    return out


def per_iteration(cases, warm_iters: int, timed_iters: int, eig_form: int = 0):
    """ms per iteration of sos_step on single problems (one workgroup), after warm_iters
    iterations (warm Jacobi starts settled), in both precision forms, with the device-clock
    split by phase and the mean Jacobi sweeps per block."""
    from paper_1708_04174_amd import binding as B
    from sosgen import families as F
    out = []
    for name in cases:
        gen, desc = PER_ITER_CASES[name]
        prob = gen(F)
        for prec, pname in ((B.SOS_FP32_MIXED, "fp32"), (B.SOS_FP64, "fp64")):
            w = B.setup_problem(prob, B.sos_default_settings(precision=prec, eig_form=eig_form))
            B.sos_step(w, warm_iters)
            inf = B.sos_step(w, timed_iters)
            w.free()
            rec = {"case": name, "description": desc, "precision": pname, "iters": timed_iters,
                   "after": warm_iters, "ms_per_iter": inf["solve_ms"] / timed_iters,
                   "affine_ms_per_iter": inf["affine_ms"] / timed_iters,
                   "projection_ms_per_iter": inf["eig_ms"] / timed_iters, "sweeps": inf["eig_sweeps"]}
            log(f"[per-iter] {name} {pname}: {rec['ms_per_iter']:.3f} ms/iter (affine {rec['affine_ms_per_iter']:.3f}, "
                f"projection {rec['projection_ms_per_iter']:.3f}, {rec['sweeps']:.1f} sweeps)")
            out.append(rec)
    return out


def _sha256(path: str) -> str:
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def _sha256_text(text: str) -> str:
    import hashlib
    return hashlib.sha256(text.encode()).hexdigest()


def measured_traffic(kernel: str, workload: str, sched):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter runs,
    or None when none were taken for this kernel and workload, or the kernel source or the
    schedule changed since they were."""
    f = os.path.join(ROOT, "profiles", "admm_mixed_lyapunov_512_traffic.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    src = _sha256(os.path.join(ROOT, "paper_1708_04174_amd", "csrc", "sos_kernels.hip"))
    sched_sha = _sha256_text(sched) if sched else None
    if rec.get("kernel") != kernel or rec.get("workload") != workload or \
            rec.get("kernel_source_sha256") != src or rec.get("schedule_sha256") != sched_sha:
        return None
    return float(rec["hbm_bytes_per_launch"])


def oracle_statuses(workload: str):
    """Stored FP64 oracle status per seed for the workload, or None if no table covers it."""
    f = os.path.join(ROOT, "tests", "golden", "oracle_tables.json")
    if not os.path.exists(f):
        return None
    tab = json.load(open(f)).get(workload)
    if not tab:
        return None
    return {int(k): int(v["status"]) for k, v in tab["seeds"].items()}


def load_schedule(name: str, override):
    """The launch schedule as a JSON string: --schedule names a file or is inline JSON."""
    if override:
        text = open(override).read() if os.path.exists(override) else override
        try:
            json.loads(text)
        except json.JSONDecodeError:
            sys.exit(f"--schedule: {override!r} is neither a JSON file nor inline JSON")
        return text
    f = os.path.join(ROOT, "paper_1708_04174_amd", "schedules", f"{name}.json")
    return open(f).read() if os.path.exists(f) else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lyapunov_512", choices=["lyapunov_512", "pop_batch_512"])
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--alpha", type=float, default=1.0, help="over-relaxation of every solve (1: the paper's steps)")
    ap.add_argument("--scale-iters", type=int, default=0,
                    help="passes of the block-scalar equilibration of every problem (0: none)")
    ap.add_argument("--schedule", default=None)
    ap.add_argument("--train-count", type=int, default=3584)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--warm-budget", type=int, default=300,
                    help="iterations a warm start may take before the solve restarts it from the cold start "
                         "(in the same launch; also at once when tau collapses)")
    ap.add_argument("--plain-sample", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-batched-fp64", action="store_true")
    ap.add_argument("--dump-infos", default=None,
                    help="write the per-problem records of the last timed step (status, iterations, "
                         "queue start / finish in ms) to this JSON file")
    ap.add_argument("--per-iter", nargs="*", default=None, metavar="CASE",
                    help="only time sos_step per iteration on single problems (cases: "
                         + ", ".join(PER_ITER_CASES) + "; none given: all) and print them as one JSON line")
    ap.add_argument("--eig-form", type=int, default=0,
                    help="--per-iter only: the eigensolver form of the single solves (sos_settings.eig_form; "
                         "0 = the library's choice, 2 = one workgroup for every block)")
    ap.add_argument("--table2", nargs="*", type=int, default=None, metavar="N",
                    help="only solve Table II's local Lyapunov programs at these n (default: Table II's sizes) "
                         "in FP64 at --tol and print them as one JSON line")
    ap.add_argument("--table1", nargs="*", type=int, default=None, metavar="N",
                    help="only solve the paper's test POP at these n (default: Table I's sizes) in FP64 at "
                         "--tol (use 1e-3, the paper's) and print one JSON line")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 256 MiB device buffer three times (the known-size kernel that "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: a batch would be split across GPUs by problem, "
                                   "which is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "copies": 3}), flush=True)
        return
    if args.table2 is not None:
        print(json.dumps({"table2": table2(args.table2 or sorted(TABLE2), args.tol), "tol": args.tol}), flush=True)
        return
    if args.table1 is not None:
        print(json.dumps({"table1": table1(args.table1 or sorted(TABLE1_CDCS_S), args.tol), "tol": args.tol}),
              flush=True)
        return
    if args.per_iter is not None:
        cases = args.per_iter or list(PER_ITER_CASES)
        print(json.dumps({"per_iteration": per_iteration(cases, 100, 50, args.eig_form)}), flush=True)
        return
    from paper_1708_04174_amd import binding as B
    from paper_1708_04174_amd import warmstart as W
    from paper_1708_04174_amd import workloads as WL

    lyap = args.workload == "lyapunov_512"
    t0 = time.perf_counter()
    if lyap:
        test_seeds = list(WL.LYAP_TEST)
        probs = WL.generate("lyapunov", test_seeds)
        train_seeds = list(WL.LYAP_TRAIN)[:args.train_count]
        train_probs = WL.generate("lyapunov", train_seeds) if train_seeds else []
    else:
        probs = WL.generate("pop_batch", range(512))
        train_probs = []
    log(f"[bench] generated {len(probs)} + {len(train_probs)} problems in {time.perf_counter() - t0:.1f}s")
    seeds = test_seeds if lyap else list(range(512))
    # a result counts where it is a solution or certificate the FP64 oracle agrees with
    ost = oracle_statuses(args.workload)

    def ok_status(seed, status):
        return status in OK_STATUS and (ost is None or ost.get(int(seed)) == status)

    def n_ok(infos, idx=None):
        idx = range(len(infos)) if idx is None else idx
        return int(sum(ok_status(seeds[j], inf["status"]) for j, inf in zip(idx, infos)))
    sched = load_schedule(args.workload, args.schedule)
    st = B.sos_default_settings(tol=args.tol, max_iters=2000, check_every=10, alpha=args.alpha, scale_iters=args.scale_iters,
                                precision=B.SOS_FP32_MIXED, polish_iters=1)
    t0 = time.perf_counter()
    works = [B.setup_problem(p, st) for p in probs]
    t_setup = time.perf_counter() - t0
    batch = B.sos_batch_setup(works, sched)
    t_bsetup = time.perf_counter() - t0 - t_setup
    layout = B.sos_layout_size(works[0])
    gpu_setup = {"ms_per_problem": 1e3 * t_setup / len(probs), "batch_setup_ms": 1e3 * t_bsetup,
                 "note": "sos_setup on the host (validation, partition, S and its inverse, h) plus the upload, "
                         "then sos_batch_setup; outside the timed step, like the oracle's set-up"}
    log(f"[bench] setup {t_setup:.1f}s + batch {t_bsetup:.1f}s")

    # ---------------------------------------------------------------- warm-start model (untimed)
    model, train_info = None, None
    if lyap and train_probs:
        t0 = time.perf_counter()
        X, T = [], []
        nsolved = 0
        for i in range(0, len(train_probs), 512):
            chunk = train_probs[i:i + 512]
            tw = [B.setup_problem(p, st) for p in chunk]
            infos, sol, tb = W.cold_solve_batch(tw, sched)
            keep = [j for j, inf in enumerate(infos) if inf["status"] == B.SOS_SOLVED]
            X.append(WL.lyapunov_features([train_seeds[i + j] for j in keep]))
            T.append(sol.cpu().numpy()[keep])   # host copy: row selection is data preparation
            nsolved = nsolved + len(keep)
            tb.free()
            for w in tw:
                w.free()
            log(f"[bench] training data {i + len(chunk)}/{len(train_probs)}: {len(keep)} solved")
        Xtr, Ttr = np.concatenate(X), np.concatenate(T)
        rows = np.nonzero(W.training_mask(Ttr))[0]
        log(f"[bench] training set: {len(rows)} of {nsolved} solved instances (norm <= 3 x median)")
        t1 = time.perf_counter()
        model = W.WarmStartModel(Xtr.shape[1], Ttr.shape[1], hidden=512, max_batch=4096, seed=0)
        losses = model.fit(Xtr, Ttr, rows=rows, epochs=args.epochs, batch=256, lr=1e-3, log=log)
        train_info = {"instances": int(len(rows)), "epochs": args.epochs, "final_loss": losses[-1],
                      "data_s": t1 - t0, "fit_s": time.perf_counter() - t1}
        log(f"[bench] model: {train_info}")
        Xte = torch.from_numpy(WL.lyapunov_features(test_seeds)).cuda()
        st_warm = B.sos_default_settings(tol=args.tol, max_iters=2000, check_every=10, alpha=args.alpha, scale_iters=args.scale_iters,
                                         precision=B.SOS_FP32_MIXED, polish_iters=1, warm_budget=args.warm_budget)
        warm_works = [B.setup_problem(p, st_warm) for p in probs]
        warm_batch = B.sos_batch_setup(warm_works, sched)

    # ---------------------------------------------------------------- cold batched (ablation)
    def cold_step():
        B.sos_batch_reset(batch)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = B.sos_batch_solve(batch)
        torch.cuda.synchronize()
        return infos, (time.perf_counter() - t) * 1e3

    cinfos, cms = cold_step()
    cold = {"value": n_ok(cinfos) / (cms / 1e3), "ms": cms,
            "iters_mean": float(np.mean([i["iters"] for i in cinfos]))}
    log(f"[bench] cold batched: {cold}")

    warm_info = {}

    def warm_step():
        B.sos_batch_reset(warm_batch)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos, nfb, _ = W.warm_solve(warm_batch, model, Xte, fallback_works=works, layout=layout, schedule=sched)
        torch.cuda.synchronize()
        warm_info["first"] = [dict(i) for i in W.LAST_FIRST_PASS]
        warm_info["fallback"] = dict(W.LAST_FALLBACK)
        return infos, (time.perf_counter() - t) * 1e3, nfb

    step = (lambda: warm_step()) if model is not None else (lambda: cold_step() + (0,))
    for i in range(args.warmup):
        _, ms, _ = step()
        log(f"[bench] warmup {i}: {ms:.1f} ms")
    step_ms, counted, kms, pms, fbs = [], [], [], [], []
    infos = None
    for i in range(args.steps):
        torch.cuda.synchronize()
        infos, ms, nfb = step()
        ok = n_ok(infos)
        step_ms.append(ms)
        counted.append(ok)
        tb = warm_batch if model is not None else batch
        kms.append(B.sos_batch_phase_ms(tb, 0))
        pms.append(B.sos_batch_phase_ms(tb, 1))
        fbs.append(nfb)
        log(f"[bench] step {i}: {ms:.1f} ms, {ok}/{len(infos)} counted, fallbacks {nfb}, "
            f"solve kernel {kms[-1]:.1f} ms, separate FP64 kernel {pms[-1]:.1f} ms")
    if args.dump_infos:
        with open(args.dump_infos, "w") as f:
            json.dump([dict(seed=int(sd), **{k: v for k, v in inf.items() if isinstance(v, (int, float, str))})
                       for sd, inf in zip(test_seeds if lyap else range(len(infos)), infos)], f)
    total_ms = float(np.sum(step_ms))
    value = float(np.sum(counted)) / (total_ms / 1e3)
    statuses = {}
    for inf in infos:
        statuses[inf["status_name"]] = statuses.get(inf["status_name"], 0) + 1
    agreement = None
    if ost is not None:
        agreement = {}
        for sd, inf in zip(seeds, infos):
            key = f"gpu_{inf['status_name']}/oracle_{B.STATUS_NAMES.get(ost[int(sd)])}"
            agreement[key] = agreement.get(key, 0) + 1
    iters = np.array([inf["iters"] for inf in infos])
    solved = [inf for inf in infos if inf["status"] == 1]
    worst = max(max(i["res_pri"], i["res_dual"], i["gap"]) for i in solved) if solved else None

    # roofline of the dominant kernel of the last step.  Mixed form in one launch
    # (admm_mixed): FP32 and FP64 iterations of every problem in the same kernel, priced
    # against the peak of each precision (the effective peak is their harmonic blend by
    # flops).  Two-launch form: the FP32 or the FP64 kernel, whichever ran longer summed
    # over the step's launches.  Figures per launch, averaged over those launches.
    first = warm_info.get("first") or infos
    fb = warm_info.get("fallback") or {}
    sched_d = json.loads(sched) if sched else {}
    thr = int(sched_d.get("block_threads", 512))

    def fl(its, idx):
        return float(sum(it * iter_flops(probs[j]) for it, j in zip(its, idx)))

    allidx = list(range(len(probs)))
    launches = []   # (ms, flops32, flops64, iterations)
    one = float(pms[-1]) == 0.0
    if one:
        kname = f"admm_mixed<{thr}>"
        parts = [(float(kms[-1]), first, allidx)]
        if fb:
            parts.append((fb["phase_ms"][0], fb["infos"], fb["idx"]))
        for ms_, inf_, idx_ in parts:
            i32 = [f["iters"] - f["polish_iters"] for f in inf_]
            i64 = [f["polish_iters"] for f in inf_]
            launches.append((ms_, fl(i32, idx_), fl(i64, idx_), int(np.sum(i32) + np.sum(i64))))
    else:
        l32 = [(float(kms[-1]), [f["iters"] - f["polish_iters"] for f in first], allidx)]
        l64 = [(float(pms[-1]), [f["polish_iters"] for f in first], allidx)]
        if fb:
            l32.append((fb["phase_ms"][0], [f["iters"] - f["polish_iters"] for f in fb["infos"]], fb["idx"]))
            l64.append((fb["phase_ms"][1], [f["polish_iters"] for f in fb["infos"]], fb["idx"]))
        if sum(x[0] for x in l32) >= sum(x[0] for x in l64):
            kname = f"admm_persistent<float, {thr}>"
            launches = [(m_, fl(i_, j_), 0.0, int(np.sum(i_))) for m_, i_, j_ in l32]
        else:
            kname = f"admm_persistent<double, {thr}>"
            launches = [(m_, 0.0, fl(i_, j_), int(np.sum(i_))) for m_, i_, j_ in l64]
    k_ms = float(np.mean([x[0] for x in launches]))
    f32 = float(np.mean([x[1] for x in launches]))
    f64 = float(np.mean([x[2] for x in launches]))
    flops = f32 + f64
    peak = flops / (f32 / PEAK_FP32_TFLOPS + f64 / PEAK_FP64_TFLOPS) if flops > 0 else PEAK_FP32_TFLOPS
    achieved = flops / (k_ms / 1e3) / 1e12 if k_ms > 0 else None
    traffic = measured_traffic(kname, args.workload, sched)
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": (achieved / peak) if achieved else None, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_GBps": (traffic / (k_ms / 1e3) / 1e9) if (traffic and k_ms > 0) else None,
                "kernel": kname, "kernel_ms": k_ms, "launches_per_step": len(launches),
                "launch_ms": [x[0] for x in launches], "algorithmic_flops_per_launch": flops,
                "fp32_flops_per_launch": f32, "fp64_flops_per_launch": f64,
                "peak_note": "FP32 157.3 and FP64 78.6 TFLOP/s vector peaks, blended by the launch's flops",
                "iterations_per_launch": float(np.mean([x[3] for x in launches]))}

    # what the learned warm start gains: iterations of the warm-started pass against the
    # cold batched solve, on the problems both solve
    warm_gain = None
    if model is not None:
        both = [i for i in range(len(probs))
                if cinfos[i]["status"] == 1 and first[i]["status"] == 1 and first[i]["warm_iters"] == 0]
        warm_gain = {"warm_budget": args.warm_budget,
                     "restarted_cold_in_launch": int(sum(f["warm_iters"] > 0 for f in first)),
                     "solved_by_warm_start": int(sum(f["status"] == 1 and f["warm_iters"] == 0 for f in first)),
                     "common_solved": len(both),
                     "cold_iters_mean": float(np.mean([cinfos[i]["iters"] for i in both])) if both else None,
                     "warm_iters_mean": float(np.mean([first[i]["iters"] for i in both])) if both else None,
                     "cold_iters_median": float(np.median([cinfos[i]["iters"] for i in both])) if both else None,
                     "warm_iters_median": float(np.median([first[i]["iters"] for i in both])) if both else None}
        log(f"[bench] warm start gain: {warm_gain}")

    plain, unbatched32 = None, None
    if not args.no_plain:
        # one problem per launch (one workgroup on one CU), cold start: every step FP64 (the
        # plain arm), and the mixed form (FP32 bulk, FP64 islands and polish) unbatched
        ns = args.plain_sample or (32 if lyap else 4)
        idx = np.linspace(0, len(probs) - 1, ns).astype(int)
        arms = {}
        for name, prec in (("fp64", B.SOS_FP64), ("fp32_mixed", B.SOS_FP32_MIXED)):
            sx = B.sos_default_settings(tol=args.tol, max_iters=2000, check_every=10, alpha=args.alpha, scale_iters=args.scale_iters, precision=prec, polish_iters=1)
            tms, okx = 0.0, 0
            for i in idx:
                w = B.setup_problem(probs[i], sx)
                inf = B.sos_solve(w)
                tms += inf["solve_ms"]
                okx += ok_status(seeds[i], inf["status"])
                w.free()
            arms[name] = {"value": okx / (tms / 1e3), "unit": "solves/s", "ms_total": tms, "counted": okx,
                          "sample": f"{len(idx)} problems spread over the workload, sos_solve one at a time, "
                                    f"{'every step FP64' if name == 'fp64' else 'FP32 bulk with FP64 islands'}, "
                                    "cold start"}
            log(f"[bench] unbatched {name}: {arms[name]['value']:.2f} solves/s")
        plain, unbatched32 = arms["fp64"], arms["fp32_mixed"]

    batched64 = None
    if not args.no_batched_fp64:
        # the whole workload in one persistent launch, every step FP64, cold start
        s64 = B.sos_default_settings(tol=args.tol, max_iters=2000, check_every=10, alpha=args.alpha, scale_iters=args.scale_iters, precision=B.SOS_FP64)
        works64 = [B.setup_problem(p, s64) for p in probs]
        batch64 = B.sos_batch_setup(works64, sched)
        b64 = []
        for rep in range(2):   # the first run captures the graph
            B.sos_batch_reset(batch64)
            torch.cuda.synchronize()
            t = time.perf_counter()
            i64 = B.sos_batch_solve(batch64)
            torch.cuda.synchronize()
            b64.append(((time.perf_counter() - t) * 1e3, i64))
        ms64, i64 = b64[-1]
        batched64 = {"value": n_ok(i64) / (ms64 / 1e3), "unit": "solves/s", "ms": ms64, "counted": n_ok(i64),
                     "iters_mean": float(np.mean([i["iters"] for i in i64])),
                     "sample": "the whole workload in one persistent launch, every step FP64, cold start"}
        log(f"[bench] batched FP64: {batched64['value']:.1f} solves/s ({ms64:.0f} ms)")
        batch64.free()
        for w in works64:
            w.free()

    cpu = None
    if not args.no_cpu_baseline:
        # the workload in a seeded random order, solved until the time budget is spent
        order = np.random.default_rng(0).permutation(len(probs))
        cpu = cpu_baseline("lyapunov" if lyap else "pop_batch", [seeds[i] for i in order], args.cpu_budget,
                           args.tol, ok_status)
        log(f"[bench] cpu baseline: {cpu['value']:.3f} solves/s on {cpu['cores']} cores ({cpu['cpu_model']})")

    desc = ("512 held-out Lyapunov programs (n = 6, quartic V: 203 free variables, Gram blocks 28 and 84, "
            "m = 1134; seeds 3584..4095), learned warm start + batched FP32 bulk / FP64 polish"
            if lyap else "512 quartic POPs (n ~ U{6..16}, Gram 28..153, m 210..4845, scaled variables; seeds 0..511), "
            "batched FP32 bulk / FP64 polish, cold start")
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "description": desc, "problems": len(probs), "tol": args.tol,
                   "alpha": args.alpha, "scale_iters": args.scale_iters,
                   "statuses": statuses, "oracle_agreement": agreement,
                   "counted_rule": "SOLVED at FP64 residual <= tol or a certificate, and the same status as the "
                                   "FP64 CPU oracle" + ("" if ost is not None else " (no oracle table: unchecked)"),
                   "iters_mean": float(iters.mean()), "iters_median": float(np.median(iters)),
                   "iters_max": int(iters.max()), "fallbacks": int(np.sum(fbs)), "worst_solved_residual": worst,
                   "phase_ms": {"solve_kernel": k_ms, "polish_kernel": float(pms[-1])},
                   "schedule": json.loads(sched) if sched else None, "warm_start_model": train_info},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "setup": {"gpu": gpu_setup, "oracle_ms_per_problem": cpu["setup_ms_per_problem"] if cpu else None},
        "plain_fp64": plain,
        "ablations": {"batched_cold_fp32": cold, "batched_fp64": batched64, "unbatched_fp32_mixed": unbatched32},
        "batched_cold_fp32": cold,
        "warm_start_gain": warm_gain,
        "speedup_vs_plain_fp64": (value / plain["value"]) if plain else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
