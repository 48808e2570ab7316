"""Pins for the oracle's solution post-processing (oracle/postprocess.py), each against
something other than the oracle: polynomial products computed by the generator's own Poly
arithmetic, closed-form decompositions, brute-force minimisers, and a planted mistake.
"""
import numpy as np
import pytest

from oracle import postprocess as PP
from oracle.admm import SOLVED, Oracle
from sosgen import Poly, families as F
from sosgen.poly import monomials


def _poly_of(prob, d2):
    """The POP's p from b over the row basis (coefficient matching puts p_alpha in b_alpha)."""
    n = prob.meta["n_vars"] if "n_vars" in prob.meta else 1
    return {e: float(v) for e, v in zip(monomials(n, d2), prob.b) if v != 0.0}, n


def test_square_sum_matches_polynomial_products():
    rng = np.random.default_rng(0)
    n = 3
    basis = monomials(n, 2)
    terms = [{e: rng.standard_normal() for e in basis} for _ in range(3)]
    ref = Poly(n)
    for q in terms:
        pq = Poly(n, q)
        ref = ref + pq * pq
    got = PP.square_sum(terms)
    keys = set(ref.terms) | set(got)
    assert max(abs(ref.terms.get(e, 0.0) - got.get(e, 0.0)) for e in keys) < 1e-12


def test_double_well_decomposes_into_one_square():
    # (x^2 - 1)^2: gamma* = 0 and X* = [[1,0,-1],[0,0,0],[-1,0,1]] = 2 v v^T, v = (1,0,-1)/sqrt(2):
    # one square, q = +-(1 - x^2)
    prob = F.univariate([1.0, 0.0, -2.0, 0.0, 1.0])
    r = Oracle.from_problem(prob).solve(tol=1e-10, max_iters=40000)
    X = r.x[1:].reshape(3, 3, order="F")
    lam, V = PP.gram_factors(X)
    assert abs(lam[0] - 2.0) < 1e-6 and np.all(lam[1:] < 1e-6)
    q = PP.sos_terms(lam[:1], V[:, :1], monomials(1, 2))[0]
    sgn = np.sign(q[(0,)])
    assert abs(sgn * q[(0,)] - 1.0) < 1e-6 and abs(q.get((1,), 0.0)) < 1e-6 and abs(sgn * q[(2,)] + 1.0) < 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_identity_residual_of_a_solved_pop(seed):
    prob = F.FAMILIES["c1"](seed)
    r = Oracle.from_problem(prob).solve(tol=1e-8, max_iters=40000)
    assert r.status == SOLVED
    N = prob.psd_dims[0]
    lam, V = PP.gram_factors(r.x[1:].reshape(N, N, order="F"))
    p, n = _poly_of(prob, 4)
    res = PP.identity_residual(p, r.x[0], PP.square_sum(PP.sos_terms(lam, V, monomials(n, 2))), n)
    # the coefficient residual is the primal residual of the certificate (A xi - b), at tol
    assert res <= 1e-8 * (1 + np.linalg.norm(prob.b)) * 10, res


def _unique_min_univariate(seed):
    rng = np.random.default_rng(seed)
    while True:
        a = np.concatenate([rng.standard_normal(4), [1.0]])      # quartic, leading coefficient 1
        crit = np.roots(np.polyder(a[::-1]))
        crit = crit[np.abs(crit.imag) < 1e-9].real
        vals = np.polyval(a[::-1], crit)
        order = np.argsort(vals)
        if len(crit) == 1 or vals[order[1]] - vals[order[0]] > 0.5:
            return a, crit[order[0]], vals[order[0]]


@pytest.mark.parametrize("seed", [3, 4])
def test_minimiser_from_moments_univariate(seed):
    a, xstar, pmin = _unique_min_univariate(seed)
    prob = F.univariate(a)
    r = Oracle.from_problem(prob).solve(tol=1e-9, max_iters=80000)
    mom = PP.moments(r.y, monomials(1, 4))
    x, ratio = PP.extract_minimiser(mom, monomials(1, 2), 1)
    assert ratio < 1e-3 and abs(x[0] - xstar) < 1e-3, (x, xstar, ratio)
    assert abs(np.polyval(a[::-1], x[0]) - pmin) < 1e-5


def test_minimiser_from_moments_bivariate():
    # p = s^2 + t^2 + s^4 + s^2 t^2 + t^4 with s = x1 - 0.5, t = x2 + 0.3: minimum 0 at (0.5, -0.3).
    # Five squares against a 6 x 6 Gram matrix (rank N - 1), so complementarity leaves a moment
    # matrix of rank one: the dual optimum is the point mass at the minimiser
    n = 2
    s = Poly.var(n, 0) - Poly.const(n, 0.5)
    t = Poly.var(n, 1) + Poly.const(n, 0.3)
    p = s * s + t * t + s * s * s * s + (s * s) * (t * t) + t * t * t * t
    prob = F.pop_from_poly(p, 2)
    r = Oracle.from_problem(prob).solve(tol=1e-9, max_iters=80000)
    assert r.status == SOLVED and abs(r.x[0]) < 1e-5
    x, ratio = PP.extract_minimiser(PP.moments(r.y, monomials(n, 4)), monomials(n, 2), n)
    assert ratio < 1e-3 and np.allclose(x, [0.5, -0.3], atol=1e-3), (x, ratio)


def test_two_minimisers_are_flagged():
    # (x^2 - 1)^2 has minimisers +-1: the moment matrix has rank two, the ratio is not small
    prob = F.univariate([1.0, 0.0, -2.0, 0.0, 1.0])
    r = Oracle.from_problem(prob).solve(tol=1e-9, max_iters=40000)
    x, ratio = PP.extract_minimiser(PP.moments(r.y, monomials(1, 4)), monomials(1, 2), 1)
    assert ratio > 0.1


def test_planted_moment_sign_mistake_is_caught():
    a, xstar, _ = _unique_min_univariate(3)
    r = Oracle.from_problem(F.univariate(a)).solve(tol=1e-9, max_iters=80000)
    # the planted version reads the moment vector mirrored (x -> -x): every odd moment flips sign
    wrong = {e: v * (-1.0 if sum(e) % 2 else 1.0) for e, v in PP.moments(r.y, monomials(1, 4)).items()}
    x, _ = PP.extract_minimiser(wrong, monomials(1, 2), 1)
    assert abs(x[0] - xstar) > 1e-2 or abs(xstar) < 1e-2
