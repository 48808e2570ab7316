"""Table II's programs (Section VII-B): local stability of a random cubic system on the ball
|x|^2 <= 0.1 with a quadratic Lyapunov function and a quadratic multiplier.

Pins, none of them the oracle checking itself:
* the generator's sizes equal the printed N, m and t of Table II at every n it lists;
* a certificate the oracle returns satisfies the three polynomial identities at random points,
  its Gram blocks are PSD and Q is positive definite, and dV/dt < 0 on sampled points of the
  ball: it proves what the program claims (lyap_cert.py, solver-free);
* a linearly unstable field (f = x) admits no certificate: primal infeasible.
"""
import numpy as np
import pytest

from lyap_cert import certificate_errors
from oracle.admm import PRIMAL_INFEASIBLE, SOLVED, Oracle
from sosgen import Poly
from sosgen import families as F

# Table II: n -> (N, m, t)
TABLE2_SHAPES = {10: (65, 1100, 110), 12: (90, 1963, 156), 14: (119, 3255, 210), 17: (170, 6273, 306),
                 20: (230, 11025, 420), 24: (324, 21050, 600), 29: (464, 41760, 870),
                 35: (665, 83475, 1260), 42: (945, 164948, 1806)}


@pytest.mark.parametrize("n", sorted(TABLE2_SHAPES))
def test_generator_matches_table2_sizes(n):
    prob = F.lyapunov_local(n, 0)
    N, m, t = TABLE2_SHAPES[n]
    assert max(prob.psd_dims) == N and prob.m == m and prob.n_free == t
    assert prob.psd_dims == [n, n, N]


@pytest.mark.parametrize("n,seed", [(3, 0), (4, 1), (5, 2)])
def test_oracle_certificate_proves_local_stability(n, seed):
    prob = F.lyapunov_local(n, seed)
    r = Oracle.from_problem(prob).solve(tol=1e-7, max_iters=20000)
    assert r.status == SOLVED
    e = certificate_errors(prob, r.x)
    print(n, seed, e)
    assert e["identity"] <= 1e-5 and e["gram_min"] >= -1e-7 and e["q_min"] > 0.0
    assert e["vdot"] <= -0.5 * prob.meta["eps"]


def test_checker_catches_a_wrong_certificate():
    # the checker itself: the same solution against a field with one term's sign flipped
    prob = F.lyapunov_local(3, 0)
    r = Oracle.from_problem(prob).solve(tol=1e-7, max_iters=20000)
    f = list(prob.meta["f"])
    f[0] = f[0] + Poly.var(3, 1).scale(-2.0 * 0.3)
    bad = dict(prob.meta, f=f)
    prob2 = F.ConicProblem(A=prob.A, b=prob.b, c=prob.c, n_free=prob.n_free, psd_dims=prob.psd_dims, meta=bad)
    assert certificate_errors(prob2, r.x)["identity"] > 1e-3


def test_unstable_field_is_primal_infeasible():
    n = 3
    prob = F.local_lyapunov_from_field(n, [Poly.var(n, i) for i in range(n)])
    r = Oracle.from_problem(prob).solve(tol=1e-6, max_iters=5000)
    assert r.status == PRIMAL_INFEASIBLE
