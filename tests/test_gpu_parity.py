"""GPU parity: the gfx950 library against the FP64 CPU oracle, through the C ABI.

Bars.  Iterates are compared entry by entry: max_i |gpu_i - ref_i| / max(1, |ref_i|).
* FP64 form: iterates after k identical steps within 1e-9 (both are exact up to rounding,
  and one ADMM step is nonexpansive, so rounding does not grow); solved objective values
  within 1e-6 relative.
* FP32 bulk (SOS_FP32_MIXED, sos_step): every step rounds the iterate to FP32 and the
  eigensolver stops at a relative coupling of 16 eps_32, so each step adds an error of a few
  hundred eps_32 times the size of the iterate; the map is nonexpansive, so after k steps the
  entries are within k * FP32_STEP_ERR * max(1, |ref|_inf) of the oracle.
* Mixed-precision solves: gamma within 5 tol relative of the FP64 oracle, and the same status.
"""
import json
import os

import numpy as np
import pytest

from oracle.admm import Oracle
from sosgen import families as F

pytestmark = pytest.mark.gpu

ITER_RTOL = 1e-9
# per-step error allowance of the FP32 bulk form, in units of the iterate's largest entry:
# 512 eps_32 (eps_32 = 1.19e-7)
FP32_STEP_ERR = 512 * 1.1920929e-07
TABLES = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_tables.json")))


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_04174_amd import binding
    binding.load()
    return binding


def _elem(a, b):
    """max_i |a_i - b_i| / max(1, |b_i|)."""
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))) if len(b) else 0.0


def _step_parity(B, prob, ks, settings=None, tag="", fp32=False):
    o = Oracle.from_problem(prob)
    w = B.setup_problem(prob, settings)
    u, v = o.initial()
    done = 0
    for k in ks:
        B.sos_step(w, k - done)
        u, v = o.run(k - done, u, v)
        done = k
        ug, vg = B.sos_get_iterate(w)
        if fp32:
            # entries relative to the iterate's largest entry (FP32 rounding is relative to it)
            scale = max(1.0, float(np.max(np.abs(u))), float(np.max(np.abs(v))))
            eu = float(np.max(np.abs(ug - u))) / scale
            ev = float(np.max(np.abs(vg - v))) / scale
            bound = k * FP32_STEP_ERR
        else:
            eu, ev = _elem(ug, u), _elem(vg, v)
            bound = ITER_RTOL
        print(f"[parity] {tag} k={k} |du|={eu:.2e} |dv|={ev:.2e} bound {bound:.1e}", flush=True)
        assert eu <= bound and ev <= bound, (tag, k, eu, ev)
    w.free()


SMALL = {
    "c1_seed0": lambda: F.FAMILIES["c1"](0),
    "univariate": lambda: F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]),
    "ball_n3_weighted": lambda: F.pop_ball(3, 2),
    "example_pop_n4": lambda: F.example_pop(4),
    "lyapunov_n2": lambda: F.lyapunov_from_field(2, F.lyapunov_field(2, np.random.default_rng(4))[2]),
    "lyapunov_c5_seed0": lambda: F.FAMILIES["c5"](0),
    # N = 55: seven column blocks, the last one partial, in the register rounds of 33 <= N <= 64
    "pop_n9": lambda: F.pop_unconstrained(9, 1),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_step_parity_small(B, name):
    _step_parity(B, SMALL[name](), [1, 2, 7, 30], tag=name)


def test_step_parity_columns_partition(B):
    # A_f = only the columns with two or more nonzeros: k = 0 for a POP, same iterates
    s = B.sos_default_settings(partition=B.SOS_PART_COLUMNS)
    _step_parity(B, F.FAMILIES["c1"](1), [1, 5, 25], settings=s, tag="c1_columns")


@pytest.mark.parametrize("threads", [64, 128, 512])
def test_step_parity_launch_shapes(B, threads):
    s = B.sos_default_settings(block_threads=threads)
    _step_parity(B, F.pop_ball(3, 4), [3, 12], settings=s, tag=f"ball3_t{threads}")


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("case", ["c5", "pop_n14"])
def test_step_parity_eigensolver_forms(B, form, case):
    # single solves: default split at N = 128, rows form for every block, lane groups for every
    # block; blocks of 28, 84 (Lyapunov) and 120 (quartic POP, n = 14)
    prob = F.FAMILIES["c5"](1) if case == "c5" else F.pop_unconstrained(14, 0)
    s = B.sos_default_settings(eig_form=form)
    _step_parity(B, prob, [1, 4, 12], settings=s, tag=f"{case}_form{form}")


def test_step_parity_c3_full_size(B):
    # constrained quartic POP on the unit ball, n = 16: Gram blocks 153 and 17, m = 4845, k = 154
    _step_parity(B, F.FAMILIES["c3"](0), [1, 3], tag="c3_full")


def test_step_parity_c2_full_size(B):
    # unconstrained quartic POP, n = 20: Gram block 231, m = 10626
    _step_parity(B, F.FAMILIES["c2"](0), [1, 2], tag="c2_full")


FP32_CASES = {
    "c1_seed0": lambda: F.FAMILIES["c1"](0),
    "ball_n3_weighted": lambda: F.pop_ball(3, 2),
    "lyapunov_c5_seed0": lambda: F.FAMILIES["c5"](0),
    "lyapunov_c5_seed3610": lambda: F.FAMILIES["c5"](3610),
    "pop_n9": lambda: F.pop_unconstrained(9, 1),
    "pop_n10": lambda: F.pop_unconstrained(10, 3),
    # N = 120: fifteen column blocks in the register rounds of 97 <= N <= 128
    "pop_n14": lambda: F.pop_unconstrained(14, 0),
    "ball_c3_full": lambda: F.FAMILIES["c3"](0),
    # blocks 105 and 14 fit in LDS together in FP32: the two-block projection with the larger
    # block's cross rounds at 16 rows per lane (97 <= N <= 128)
    "ball_n13_two_blocks": lambda: F.pop_ball(13, 0),
}


@pytest.mark.parametrize("name", list(FP32_CASES))
def test_step_parity_fp32_bulk(B, name):
    # the FP32 kernels (affine step and eigensolvers in FP32, FP64 small solve, theta and
    # tau / kappa) step by step against the FP64 oracle, at the C5 (blocks 28 + 84, k = 203)
    # and C3 (blocks 153 + 17, k = 154) shapes among others
    s = B.sos_default_settings(precision=B.SOS_FP32_MIXED)
    _step_parity(B, FP32_CASES[name](), [1, 3, 10, 30], settings=s, tag=f"fp32_{name}", fp32=True)


def test_c2_status_matches_the_oracle(B):
    # the n = 20 POP with N(0, 0.1) quartic cross terms is unbounded below, so max gamma is
    # primal infeasible: the FP64 GPU solve must end with the certificate the oracle gives
    ref = TABLES["pop_n20"]["seeds"]["0"]
    w = B.setup_problem(F.FAMILIES["c2"](0), B.sos_default_settings(tol=1e-4, max_iters=2000))
    info = B.sos_solve(w)
    print(f"[c2] gpu {info['status_name']} after {info['iters']} (oracle status {ref['status']} after "
          f"{ref['iters']}), {info['solve_ms']:.0f} ms, {info['solve_ms'] / max(1, info['iters']):.3f} ms/iter",
          flush=True)
    assert info["status"] == ref["status"] == B.SOS_PRIMAL_INFEASIBLE
    assert abs(info["iters"] - ref["iters"]) <= 20
    w.free()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c3_mixed_precision_gamma_error(B, seed):
    # constrained quartic POP on the unit ball, n = 16 (blocks 153 and 17, m = 4845, k = 154),
    # FP32 bulk / FP64 islands and polish, against the oracle's gamma at tol 1e-7
    ref = TABLES["ball_pop_n16"]["seeds"][str(seed)]
    s = B.sos_default_settings(tol=1e-4, max_iters=2000, precision=B.SOS_FP32_MIXED, polish_iters=1)
    w = B.setup_problem(F.FAMILIES["c3"](seed), s)
    info = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    g_ref = ref["reference"]["gamma"]
    err = abs(x[0] - g_ref) / max(1.0, abs(g_ref))
    res = max(info["res_pri"], info["res_dual"], info["gap"])
    print(f"[c3] seed {seed}: {info['status_name']} in {info['iters']} iterations ({info['polish_iters']} FP64), "
          f"gamma {x[0]:.6f} vs oracle {g_ref:.6f}: error {err:.2e} (bound 5e-4); res {res:.1e}; "
          f"oracle at 1e-4: status {ref['tol_1e-4']['status']} in {ref['tol_1e-4']['iters']}; "
          f"{info['solve_ms']:.0f} ms", flush=True)
    assert info["status"] == B.SOS_SOLVED == ref["tol_1e-4"]["status"] and res <= 1e-4
    assert err <= 5e-4
    w.free()


def test_c5_statuses_match_the_oracle(B):
    # the benchmark's Lyapunov programs, batched in the mixed form from the cold start: the
    # status of each (solved, primal infeasible, iteration cap) equals the oracle's, on a slice
    # that holds infeasible instances (3610, 3611) and iteration-cap ones
    table = TABLES["lyapunov_512"]["seeds"]
    seeds = list(range(3600, 3664))
    s = B.sos_default_settings(tol=1e-4, max_iters=2000, precision=B.SOS_FP32_MIXED, polish_iters=1)
    works = [B.setup_problem(F.lyapunov(sd), s) for sd in seeds]
    bt = B.sos_batch_setup(works)
    infos = B.sos_batch_solve(bt)
    bad = []
    for sd, inf in zip(seeds, infos):
        ref = table[str(sd)]
        if inf["status"] != ref["status"]:
            bad.append((sd, inf["status_name"], inf["iters"], ref["status"], ref["iters"]))
    counts = {}
    for inf in infos:
        counts[inf["status_name"]] = counts.get(inf["status_name"], 0) + 1
    print(f"[c5] statuses {counts}; disagreements with the oracle: {bad}", flush=True)
    assert {table[str(sd)]["status"] for sd in seeds} >= {1, 2}
    assert not bad
    bt.free()


CLOSED = [
    ("x_squared", lambda: F.univariate([0.0, 0.0, 1.0]), 0.0),
    ("double_well", lambda: F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]), 0.0),
]


@pytest.mark.parametrize("name,make,gamma", CLOSED)
def test_solve_closed_forms(B, name, make, gamma):
    s = B.sos_default_settings(tol=1e-9, max_iters=20000)
    w = B.setup_problem(make(), s)
    info = B.sos_solve(w)
    x, y, z = B.sos_get_solution(w)
    print(f"[solve] {name} status={info['status_name']} iters={info['iters']} gamma={x[0]:.3e}", flush=True)
    assert info["status"] == B.SOS_SOLVED and abs(x[0] - gamma) < 1e-6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solve_parity_c1(B, seed):
    prob = F.FAMILIES["c1"](seed)
    r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=20000, check_every=10)
    s = B.sos_default_settings(tol=1e-6, max_iters=20000, check_every=10)
    w = B.setup_problem(prob, s)
    info = B.sos_solve(w)
    x, y, z = B.sos_get_solution(w)
    print(f"[solve] c1 seed={seed} gpu iters={info['iters']} gamma={x[0]:.9f} oracle iters={r.iters} "
          f"gamma={r.x[0]:.9f}", flush=True)
    assert info["status"] == B.SOS_SOLVED and r.status == 1
    assert info["iters"] == r.iters
    assert abs(x[0] - r.x[0]) <= 1e-6 * max(1.0, abs(r.x[0]))
    assert max(info["res_pri"], info["res_dual"], info["gap"]) <= 1e-6


def test_solve_status_certificates(B):
    for make, status in ((F.infeasible_pop, B.SOS_PRIMAL_INFEASIBLE), (F.unbounded_pop, B.SOS_DUAL_INFEASIBLE)):
        prob = make()
        r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=5000)
        w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=5000))
        info = B.sos_solve(w)
        print(f"[solve] {prob.meta['family']} gpu={info['status_name']} oracle={r.status_name}", flush=True)
        assert info["status"] == status == r.status and info["iters"] == r.iters


def test_checkpoint_resume(B):
    # the method's state is (u, v): k1 steps, save, restore into a fresh handle, k2 steps
    # equals k1 + k2 steps straight.  The restored handle's eigensolver starts without the
    # cached eigenvectors, so only rounding differs; the round trip of the state is exact.
    prob = F.pop_ball(3, 7)
    w1 = B.setup_problem(prob)
    B.sos_step(w1, 17)
    u_mid, v_mid = B.sos_get_iterate(w1)
    B.sos_step(w1, 23)
    u_ref, v_ref = B.sos_get_iterate(w1)
    w2 = B.setup_problem(prob)
    B.sos_set_iterate(w2, u_mid, v_mid)
    u_back, v_back = B.sos_get_iterate(w2)
    assert np.array_equal(u_back, u_mid) and np.array_equal(v_back, v_mid)
    B.sos_step(w2, 23)
    u2, v2 = B.sos_get_iterate(w2)
    assert _elem(u2, u_ref) <= 1e-12 and _elem(v2, v_ref) <= 1e-12


def test_repeat_runs_are_bitwise_equal(B):
    prob = F.FAMILIES["c5"](3)
    outs = []
    for _ in range(2):
        w = B.setup_problem(prob)
        B.sos_step(w, 25)
        outs.append(B.sos_get_iterate(w))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_setup_errors(B):
    prob = F.FAMILIES["c1"](0)
    A = prob.A.tolil(copy=True)
    N = prob.psd_dims[0]
    A[0, 1 + 1 * N + 0] = A[0, 1 + 1 * N + 0] + 1.0      # break the (i,j)/(j,i) symmetry
    with pytest.raises(B.SosError) as e:
        B.sos_setup(A.tocsc(), prob.b, prob.c, prob.n_free, prob.psd_dims)
    assert e.value.code == B.SOS_E_ASYM
    with pytest.raises(B.SosError) as e:
        B.sos_setup(prob.A, prob.b, prob.c, prob.n_free, [N + 1])
    assert e.value.code == B.SOS_E_INVAL
    bad = prob.b.copy()
    bad[3] = np.nan
    with pytest.raises(B.SosError) as e:
        B.sos_setup(prob.A, bad, prob.c, prob.n_free, prob.psd_dims)
    assert e.value.code == B.SOS_E_INVAL


def test_settings_and_schedule_errors(B):
    prob = F.FAMILIES["c1"](0)
    with pytest.raises(B.SosError) as e:
        B.setup_problem(prob, B.sos_default_settings(eig_form=4))
    assert e.value.code == B.SOS_E_INVAL
    works = [B.setup_problem(F.pop_unconstrained(4, sd)) for sd in (0, 1)]
    for bad in ('{"eig_wave": 1}', '{"rows_nmin": -1}', '{"stall_checks": 0}', '{"fp64_jacobi_tol": 0.01}',
                '{"gs_n64": 12}', '{"block_threads": 96}', '{"lds_kb": 400}'):
        with pytest.raises(B.SosError) as e:
            B.sos_batch_setup(works, bad)
        assert e.value.code == B.SOS_E_INVAL, bad
    # the handles are untouched by the refused schedules
    bt = B.sos_batch_setup(works, '{"eig_wave": 2, "rows_nmin": 0, "stall_checks": 8, "fp64_jacobi_tol": 0}')
    infos = B.sos_batch_solve(bt)
    assert all(i["status"] == B.SOS_SOLVED for i in infos)
    bt.free()


def test_batch_queue_stamps(B):
    # each problem's queue start and finish lie inside the launch, start <= finish; single
    # solves report zeros
    probs = [F.pop_unconstrained(n, sd) for n, sd in ((4, 0), (5, 1), (6, 2))] + [F.FAMILIES["c5"](2)]
    s = B.sos_default_settings(precision=B.SOS_FP32_MIXED, polish_iters=1)
    works = [B.setup_problem(p, s) for p in probs]
    bt = B.sos_batch_setup(works, '{"use_graph": 0}')
    infos = B.sos_batch_solve(bt)
    launch = B.sos_batch_phase_ms(bt, 0)
    for inf in infos:
        print(f"[stamps] start {inf['start_ms']:.3f} end {inf['end_ms']:.3f} launch {launch:.3f}", flush=True)
        assert 0.0 <= inf["start_ms"] <= inf["end_ms"] <= launch + 1e-6
    assert min(i["start_ms"] for i in infos) < 1.0
    bt.free()
    w = B.setup_problem(probs[0], s)
    inf = B.sos_solve(w)
    assert inf["start_ms"] == 0.0 and inf["end_ms"] == 0.0
    w.free()


def test_batch_fp64_equals_single_solves(B):
    # one persistent launch over uneven problems gives the same iterates as one launch per problem
    probs = [F.pop_unconstrained(n, sd) for n, sd in ((4, 0), (5, 1), (6, 2), (7, 3), (8, 4))]
    probs += [F.pop_ball(3, 1), F.FAMILIES["c5"](1)]
    s = B.sos_default_settings(tol=1e-5, max_iters=3000)
    singles = []
    for p in probs:
        print(f"[batch] single solve N={p.psd_dims}", flush=True)
        w = B.setup_problem(p, s)
        inf = B.sos_solve(w)
        singles.append((inf, B.sos_get_iterate(w)))
        w.free()
    works = [B.setup_problem(p, s) for p in probs]
    bt = B.sos_batch_setup(works, '{"wg_per_cu": 1}')
    infos = B.sos_batch_solve(bt)
    for (inf1, (u1, v1)), inf2, w in zip(singles, infos, works):
        u2, v2 = B.sos_get_iterate(w)
        print(f"[batch] {inf1['status_name']} iters {inf1['iters']} vs {inf2['iters']}", flush=True)
        assert inf1["status"] == inf2["status"] and inf1["iters"] == inf2["iters"]
        assert np.array_equal(u1, u2) and np.array_equal(v1, v2)
    # a second solve of the same batch from the cold start repeats the first exactly
    B.sos_batch_reset(bt)
    infos2 = B.sos_batch_solve(bt)
    assert [i["iters"] for i in infos2] == [i["iters"] for i in infos]
    bt.free()


def test_batch_mixed_precision_gamma_error(B):
    # FP32 bulk + FP64 polish: the status equals the oracle's at the same tolerance and
    # iteration budget, and a solved gamma is within 5 tol of the oracle's tol 1e-7 value.
    # The n = 6 and n = 7 POPs (seeds 5, 6) sit at the edge of SOS feasibility: the oracle
    # itself does not reach 1e-4 within the budget, and neither does the GPU
    probs = [F.pop_unconstrained(n, sd) for n, sd in ((4, 0), (4, 1), (4, 3), (5, 4), (6, 5), (7, 6))]
    probs += [F.pop_ball(3, 5)]
    s = B.sos_default_settings(tol=1e-4, max_iters=4000, precision=B.SOS_FP32_MIXED, polish_iters=1)
    works = [B.setup_problem(p, s) for p in probs]
    bt = B.sos_batch_setup(works)
    infos = B.sos_batch_solve(bt)
    for p, inf, w in zip(probs, infos, works):
        o = Oracle.from_problem(p)
        same = o.solve(tol=1e-4, max_iters=4000)
        res = max(inf["res_pri"], inf["res_dual"], inf["gap"])
        line = (f"[mixed] N={p.psd_dims} status={inf['status_name']} iters={inf['iters']} "
                f"(fp64 {inf['polish_iters']}) res {res:.1e}; oracle {same.status_name} in {same.iters}")
        assert inf["status"] == same.status, line
        if same.status == 1:
            r = o.solve(tol=1e-7, max_iters=30000)
            x, _, _ = B.sos_get_solution(w)
            err = abs(x[0] - r.x[0]) / max(1.0, abs(r.x[0]))
            line += f"; gamma err {err:.2e}"
            assert res <= 1e-4 and err <= 5e-4, line
        print(line, flush=True)
    bt.free()


def test_single_mixed_precision_solve(B):
    prob = F.pop_ball(3, 6)
    r = Oracle.from_problem(prob).solve(tol=1e-7, max_iters=30000)
    w = B.setup_problem(prob, B.sos_default_settings(tol=1e-4, precision=B.SOS_FP32_MIXED))
    inf = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    print(f"[mixed] single status={inf['status_name']} iters={inf['iters']} polish={inf['polish_iters']} "
          f"gamma {x[0]:.6f} vs {r.x[0]:.6f}", flush=True)
    assert inf["status"] == B.SOS_SOLVED and inf["polish_iters"] >= 1
    assert abs(x[0] - r.x[0]) <= 5e-4 * max(1.0, abs(r.x[0]))


@pytest.mark.parametrize("sched", ['{}', '{"eig_wave": 2, "rows_nmin": 0}',
                                   '{"eig_wave": 0, "gs_n32": 8, "gs_n64": 32}',
                                   '{"eig_wave": 0, "gs_n32": 16, "gs_n64": 8}',
                                   '{"eig_wave": 2, "rows_nmin": 0, "block_threads": 256, "wg_per_cu": 2}'])
def test_batch_eigensolver_forms_match_the_oracle(B, sched):
    # every eigensolver form a schedule can pick (rows over the wavefronts, lane groups
    # of 8, 16 or 32 per column pair) gives the oracle's gamma and status (FP64)
    probs = [F.pop_unconstrained(n, sd) for n, sd in ((4, 0), (5, 1), (6, 2))] + [F.pop_ball(3, 1)]
    s = B.sos_default_settings(tol=1e-6, max_iters=4000)
    works = [B.setup_problem(p, s) for p in probs]
    bt = B.sos_batch_setup(works, sched)
    infos = B.sos_batch_solve(bt)
    for p, inf, w in zip(probs, infos, works):
        r = Oracle.from_problem(p).solve(tol=1e-6, max_iters=4000)
        x, _, _ = B.sos_get_solution(w)
        err = abs(x[0] - r.x[0]) / max(1.0, abs(r.x[0]))
        print(f"[forms] {sched} N={p.psd_dims} {inf['status_name']} iters {inf['iters']} (oracle {r.iters}) "
              f"gamma err {err:.1e}", flush=True)
        assert inf["status"] == r.status and err <= 1e-6
    bt.free()


def test_autotuner_writes_a_schedule_the_batch_accepts(B):
    import json

    from paper_1708_04174_amd import autotune
    probs = [F.pop_unconstrained(n, sd) for n, sd in ((4, 0), (5, 1), (6, 2), (7, 3))]
    sched = autotune.tune(probs, B.SOS_FP32_MIXED, iters=10, sample=4, log=lambda m: print(m, flush=True))
    for k in ("block_threads", "wg_per_cu", "eig_wave", "rows_nmin", "gs_n32", "use_graph"):
        assert k in sched
    # the tuned schedule changes speed, not answers: statuses as with the default schedule,
    # gamma within the mixed-precision bound
    st = B.sos_default_settings(tol=1e-4, precision=B.SOS_FP32_MIXED)
    out = []
    for sc in (None, json.dumps(sched)):
        works = [B.setup_problem(p, st) for p in probs]
        bt = B.sos_batch_setup(works, sc)
        infos = B.sos_batch_solve(bt)
        gam = [B.sos_get_solution(w)[0][0] if i["status"] == B.SOS_SOLVED else None for i, w in zip(infos, works)]
        out.append(([i["status"] for i in infos], gam))
        bt.free()
    print(f"[tune] statuses default {out[0][0]} tuned {out[1][0]}", flush=True)
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        if a is not None:
            assert abs(a - b) <= 5e-4 * max(1.0, abs(a))


def test_mixed_one_launch_equals_two_launches(B):
    # the mixed form in one launch (each problem widens to FP64 as soon as its own FP32
    # phase ends) computes exactly what the two-launch form does
    probs = [F.pop_unconstrained(n, sd) for n, sd in ((4, 0), (4, 1), (5, 4))] + [F.pop_ball(3, 5), F.lyapunov(3)]
    s = B.sos_default_settings(tol=1e-4, max_iters=2000, precision=B.SOS_FP32_MIXED, polish_iters=1)
    res = []
    for one in (1, 0):
        works = [B.setup_problem(p, s) for p in probs]
        bt = B.sos_batch_setup(works, f'{{"one_launch": {one}}}')
        infos = B.sos_batch_solve(bt)
        res.append(([(i["status"], i["iters"], i["polish_iters"]) for i in infos], [B.sos_get_iterate(w) for w in works]))
        print(f"[mixed] one_launch={one}: {res[-1][0]}; launch {B.sos_batch_phase_ms(bt, 0):.1f} + "
              f"{B.sos_batch_phase_ms(bt, 1):.1f} ms", flush=True)
        bt.free()
    assert res[0][0] == res[1][0]
    for (u1, v1), (u2, v2) in zip(res[0][1], res[1][1]):
        assert np.array_equal(u1, u2) and np.array_equal(v1, v2)


# ---------------------------------------------------------------- multi-workgroup (cooperative) form
COOP_CASES = {
    "c1_seed0": lambda: F.FAMILIES["c1"](0),                 # one block of 15: a single column block pair
    "lyapunov_c5_seed0": lambda: F.FAMILIES["c5"](0),        # blocks 84 and 28, k = 203
    "ball_n3_weighted": lambda: F.pop_ball(3, 2),             # blocks 10 and 4
    "pop_n14": lambda: F.pop_unconstrained(14, 0),            # block 120: 15 column blocks (odd)
}


@pytest.mark.parametrize("name", list(COOP_CASES))
def test_step_parity_multi_workgroup(B, name):
    # eig_form 3: every block through the cooperative grid (block Jacobi, grid barriers)
    s = B.sos_default_settings(eig_form=3)
    _step_parity(B, COOP_CASES[name](), [1, 3, 12], settings=s, tag=f"{name}_coop")


def test_solve_parity_multi_workgroup(B):
    for seed in (0, 1):
        prob = F.FAMILIES["c1"](seed)
        r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=5000)
        w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=5000, eig_form=3))
        inf = B.sos_solve(w)
        x, _, _ = B.sos_get_solution(w)
        w.free()
        print(f"[parity] coop c1 seed {seed}: gpu {inf['status_name']} {inf['iters']} gamma {x[0]:.9f}; "
              f"oracle {r.status_name} {r.iters} gamma {r.x[0]:.9f}", flush=True)
        assert inf["status"] == r.status == 1 and inf["iters"] == r.iters
        assert abs(x[0] - r.x[0]) <= 1e-6 * max(1.0, abs(r.x[0]))


def test_example_pop_n24_through_sos_solve(B):
    # the paper's test POP (Section VII-A) at n = 24: blocks 325 and 25, m = 20475 (Table I's
    # n = 24 row); FP64 on the multi-workgroup form, against the oracle's stored solve
    ref = TABLES["example_pop_n24"]
    prob = F.example_pop(24)
    assert prob.psd_dims == [325, 25] and prob.m == 20475
    w = B.setup_problem(prob, B.sos_default_settings(tol=ref["tol"], max_iters=ref["max_iters"]))
    inf = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    w.free()
    o = ref["result"]
    print(f"[parity] example POP n = 24: gpu {inf['status_name']} {inf['iters']} gamma {x[0]:.9f} "
          f"({inf['solve_ms'] / max(inf['iters'], 1):.2f} ms/iter, {inf['eig_sweeps']:.1f} sweeps); "
          f"oracle {o['status']} {o['iters']} gamma {o['gamma']:.9f}", flush=True)
    assert inf["status"] == o["status"] == 1 and inf["iters"] == o["iters"]
    assert abs(x[0] - o["gamma"]) <= 1e-6 * abs(o["gamma"])


@pytest.mark.parametrize("form", [0, 2])
def test_step_parity_wide_lowrank_part(B, form):
    # ball POP n = 8 at 2d = 6: Gram blocks 165 and 45, the weighted block's 1035 lower-triangle
    # columns in A_f (k = 1036, past the LDS k-vector); the multi-workgroup and one-workgroup forms
    prob = F.pop_ball(8, 0, form="weighted", half_degree=3)
    assert prob.psd_dims == [165, 45]
    s = B.sos_default_settings(eig_form=form)
    w = B.setup_problem(prob, s)
    assert B.sos_step(w, 0)["k_lowrank"] == 1036
    w.free()
    _step_parity(B, prob, [1, 3], settings=s, tag=f"ball_n8_2d6_form{form}")


def test_many_blocks_step_and_solve(B):
    # ten Gram blocks in one program (past the former limit of eight)
    rng = np.random.default_rng(400)
    polys = [np.concatenate([rng.standard_normal(4), [1.0]]) for _ in range(10)]
    prob = F.univariate_stack(polys)
    _step_parity(B, prob, [1, 5, 40], tag="univariate_stack_10")
    r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=20000)
    w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=20000))
    inf = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    w.free()
    assert inf["status"] == r.status == 1 and inf["iters"] == r.iters
    assert np.max(np.abs(x[:10] - r.x[:10])) <= 1e-6 * max(1.0, np.max(np.abs(r.x[:10])))


def test_cached_eigenvectors_stay_orthogonal(B):
    # the FP32 bulk iterations rotate the cached eigenvectors with hardware reciprocal square roots
    # (c^2 + s^2 = 1 to a few ulp) and never re-orthonormalise them: measure ||V^T V - I||_max of
    # the Lyapunov program's blocks (84 and 28) after 50 and 500 warm FP32 iterations
    prob = F.FAMILIES["c5"](0)
    w = B.setup_problem(prob, B.sos_default_settings(precision=B.SOS_FP32_MIXED))
    errs = {}
    done = 0
    for k in (50, 500):
        B.sos_step(w, k - done)
        done = k
        for b in range(len(prob.psd_dims)):
            V, valid = B.sos_get_eig_cache(w, b, B.SOS_FP32_MIXED)
            assert valid
            errs[(k, b)] = float(np.max(np.abs(V.T @ V - np.eye(V.shape[0]))))
    w.free()
    print(f"[parity] cached eigenvector orthogonality (FP32): {errs}", flush=True)
    # FP32 columns are orthonormal to about N eps_32 after one rebuild; drift stays within 1e-4
    assert max(errs.values()) <= 1e-4


def test_multi_workgroup_runs_are_bitwise_equal(B):
    # the grid-wide affine step and the Gram-based block rounds sum in fixed orders: two solves of
    # the same problem on the cooperative form give the same bits
    prob = F.example_pop(16)
    outs = []
    for _ in range(2):
        w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=3000, eig_form=3))
        inf = B.sos_solve(w)
        u, v = B.sos_get_iterate(w)
        V, valid = B.sos_get_eig_cache(w, 0, B.SOS_FP64)
        w.free()
        outs.append((inf["iters"], u, v))
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])
    # the cached FP64 eigenvectors of the cooperative form stay orthonormal to rounding (they are
    # rotated by products with the blocks' 16 x 16 rotations and never re-orthonormalised)
    orth = float(np.max(np.abs(V.T @ V - np.eye(V.shape[0]))))
    print(f"[parity] multi-workgroup: {outs[0][0]} iterations twice, cached V orthogonality {orth:.2e}", flush=True)
    assert valid and orth <= 1e-10
