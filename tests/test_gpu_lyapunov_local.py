"""Table II's programs (Section VII-B) on the GPU, through the C ABI: step parity with the FP64
oracle, solves whose certificates are checked without any solver (lyap_cert.py), the infeasible
case, and a large instance on the multi-workgroup form."""
import numpy as np
import pytest

from lyap_cert import certificate_errors
from oracle.admm import Oracle
from sosgen import Poly
from sosgen import families as F

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_04174_amd import binding
    binding.load()
    return binding


def _elem(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


@pytest.mark.parametrize("n", [4, 10])
def test_step_parity(B, n):
    # blocks n, n and C(n+2, 2) - 1; t = n (n + 1) free columns; FP64 iterates within 1e-9
    prob = F.lyapunov_local(n, 3)
    o = Oracle.from_problem(prob)
    w = B.setup_problem(prob)
    u, v = o.initial()
    done = 0
    for k in (1, 5, 20):
        B.sos_step(w, k - done)
        u, v = o.run(k - done, u, v)
        done = k
        ug, vg = B.sos_get_iterate(w)
        eu, ev = _elem(ug, u), _elem(vg, v)
        print(f"[parity] lyapunov_local n={n} k={k} |du|={eu:.2e} |dv|={ev:.2e}", flush=True)
        assert eu <= 1e-9 and ev <= 1e-9
    w.free()


@pytest.mark.parametrize("n,precision", [(4, "fp64"), (10, "fp64"), (10, "mixed")])
def test_solve_certificate(B, n, precision):
    prob = F.lyapunov_local(n, 5)
    prec = B.SOS_FP64 if precision == "fp64" else B.SOS_FP32_MIXED
    w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=5000, precision=prec))
    inf = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    w.free()
    r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=5000)
    e = certificate_errors(prob, x)
    print(f"[parity] lyapunov_local n={n} {precision}: gpu {inf['status_name']} {inf['iters']}, "
          f"oracle {r.status_name} {r.iters}; certificate {e}", flush=True)
    assert inf["status"] == r.status == 1
    if precision == "fp64":
        assert inf["iters"] == r.iters
    assert e["identity"] <= 1e-4 and e["gram_min"] >= -1e-6 and e["q_min"] > 0.0
    assert e["vdot"] <= -0.5 * prob.meta["eps"]


def test_unstable_field_is_primal_infeasible(B):
    n = 4
    prob = F.local_lyapunov_from_field(n, [Poly.var(n, i) for i in range(n)])
    w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=5000))
    inf = B.sos_solve(w)
    w.free()
    r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=5000)
    assert inf["status"] == r.status == B.SOS_PRIMAL_INFEASIBLE


def test_table2_n24_certificate(B):
    # Table II's n = 24 row: blocks 24, 24, 324, m = 21050, t = 600; FP64 multi-workgroup form
    # for the N = 324 block; the certificate is checked by the solver-free checker
    prob = F.lyapunov_local(24, 0)
    assert prob.psd_dims == [24, 24, 324] and prob.m == 21050 and prob.n_free == 600
    w = B.setup_problem(prob, B.sos_default_settings(tol=1e-6, max_iters=2000))
    inf = B.sos_solve(w)
    x, _, _ = B.sos_get_solution(w)
    w.free()
    e = certificate_errors(prob, x, samples=100)
    print(f"[parity] lyapunov_local n=24: {inf['status_name']} in {inf['iters']} iterations, "
          f"{inf['solve_ms'] / max(inf['iters'], 1):.2f} ms/iter; certificate {e}", flush=True)
    assert inf["status"] == B.SOS_SOLVED
    assert e["identity"] <= 1e-4 and e["gram_min"] >= -1e-6 and e["q_min"] > 0.0
    assert e["vdot"] <= -0.5 * prob.meta["eps"]
