"""Pins for the oracle's convergence variants, each against something other than the oracle.

* Over-relaxation (alpha in (1, 2)): a solution of the embedding is still a fixed point, and
  relaxed solves reach the closed forms and brute-force minima; certificates are still found.
* Block-scalar equilibration (row scaling D, one column factor per PSD block): D A E keeps
  partial orthogonality (Proposition 1) and the cone; Ruiz's fixed point equilibrates the
  rows and the blocks; the solution returned in the original units satisfies the original
  problem (checked here with A, b, c directly); closed forms are still reached.
* Planted mistakes in copies of the oracle that these pins catch.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.admm import (DUAL_INFEASIBLE, PRIMAL_INFEASIBLE, SOLVED, Oracle,
                         block_scalar_equilibration)
from sosgen import families as F

ALPHA = 1.6


def _brute_univariate(a):
    crit = np.roots(np.polyder(a[::-1]))
    crit = crit[np.abs(crit.imag) < 1e-9].real
    return min(np.polyval(a[::-1], crit))


def _converged_state(o, prob_tol=1e-11):
    r = o.solve(tol=prob_tol, max_iters=40000)
    n, m = o.n, o.m
    u = np.concatenate([r.x, r.y, [1.0]])
    v = np.concatenate([r.z, np.zeros(m), [0.0]])
    return o.rescale(u, v)


# ---------------------------------------------------------------- over-relaxation
def test_relaxed_step_keeps_a_solution_fixed():
    # at a fixed point the affine step returns u itself, so alpha u_hat + (1 - alpha) u = u
    o = Oracle.from_problem(F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]))
    u, v = _converged_state(o)
    u2, v2 = o.step(u, v, alpha=ALPHA)
    assert np.linalg.norm(u2 - u) < 1e-7 and np.linalg.norm(v2 - v) < 1e-7


def test_relaxed_solves_reach_closed_forms():
    r = Oracle.from_problem(F.univariate([0.0, 0.0, 1.0])).solve(tol=1e-9, max_iters=20000, alpha=ALPHA)
    assert r.status == SOLVED and abs(r.x[0]) < 1e-6
    r = Oracle.from_problem(F.univariate([1.0, 0.0, -2.0, 0.0, 1.0])).solve(tol=1e-9, max_iters=20000, alpha=ALPHA)
    assert r.status == SOLVED and abs(r.x[0]) < 1e-6
    X = r.x[1:].reshape(3, 3, order="F")
    assert np.allclose(X, [[1, 0, -1], [0, 0, 0], [-1, 0, 1]], atol=1e-5)


@pytest.mark.parametrize("seed", [0, 1])
def test_relaxed_univariate_bound_equals_brute_force_minimum(seed):
    rng = np.random.default_rng(200 + seed)
    a = np.concatenate([rng.standard_normal(6), [1.0]])
    pmin = _brute_univariate(a)
    r = Oracle.from_problem(F.univariate(a)).solve(tol=1e-8, max_iters=50000, alpha=ALPHA)
    assert r.status == SOLVED and abs(r.x[0] - pmin) <= 1e-5 * max(1.0, abs(pmin))


def test_relaxed_certificates():
    assert Oracle.from_problem(F.infeasible_pop()).solve(tol=1e-6, max_iters=5000, alpha=ALPHA).status == \
        PRIMAL_INFEASIBLE
    assert Oracle.from_problem(F.unbounded_pop()).solve(tol=1e-6, max_iters=5000, alpha=ALPHA).status == \
        DUAL_INFEASIBLE


class _RelaxTowardV(Oracle):
    """Planted mistake: the relaxation mixes in v instead of u."""
    def step(self, u, v, alpha=1.0):
        u_hat = self.affine(u + v)
        u_hat = alpha * u_hat + (1.0 - alpha) * v
        u_new = self.project_C(u_hat - v)
        return u_new, v - u_hat + u_new


def test_planted_relaxation_mistake_is_caught():
    good = Oracle.from_problem(F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]))
    u, v = _converged_state(good)
    bad = _RelaxTowardV.from_problem(F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]))
    u2, v2 = bad.step(u, v, alpha=ALPHA)
    assert np.linalg.norm(u2 - u) + np.linalg.norm(v2 - v) > 1e-3


# ---------------------------------------------------------------- equilibration
CASES = {
    "c1": lambda: F.FAMILIES["c1"](0),
    "ball3_weighted": lambda: F.pop_ball(3, 2),
    "lyap_c5": lambda: F.FAMILIES["c5"](0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_equilibration_keeps_partial_orthogonality_and_the_cone(name):
    prob = CASES[name]()
    A = sp.csc_matrix(prob.A)
    D, E = block_scalar_equilibration(A, prob.n_free, prob.psd_dims, 10)
    assert np.all(D > 0) and np.all(E > 0)
    off = prob.n_free
    for N in prob.psd_dims:
        blk = E[off:off + N * N]
        assert np.all(blk == blk[0])                 # one factor per PSD block: the cone is kept
        off += N * N
    S = sp.csc_matrix(sp.diags(D) @ A @ sp.diags(E))
    nnz = np.diff(A.indptr)
    single = np.where(nnz == 1)[0]
    single = single[single >= prob.n_free]           # the PSD columns with one nonzero
    As = S[:, single]
    G = (As @ As.T).toarray()
    assert np.allclose(G, np.diag(np.diag(G)), atol=0.0)    # A_s A_s^T still exactly diagonal


@pytest.mark.parametrize("name", list(CASES))
def test_equilibration_equalises_rows_and_column_groups(name):
    # the passes converge to D A E whose nonzero rows share one 2-norm and whose column groups
    # (each free variable, each PSD block) share one root-mean-square column norm, with the row
    # scaling balanced (geometric mean 1); the unscaled matrix has neither property
    prob = CASES[name]()
    A = sp.csc_matrix(prob.A)

    def spreads(D, E):
        S = sp.csr_matrix(sp.diags(D) @ A @ sp.diags(E))
        rows = np.sqrt(np.asarray(S.multiply(S).sum(axis=1)).ravel())
        rows = rows[(D > 1e-4) & (D < 1e4)]          # rows whose factor sits at a clamp are apart
        cols2 = np.asarray(S.multiply(S).sum(axis=0)).ravel()
        grp = [np.sqrt(cols2[j]) for j in range(prob.n_free)]
        off = prob.n_free
        for N in prob.psd_dims:
            grp.append(np.sqrt(cols2[off:off + N * N].mean()))
            off += N * N
        rows, grp = rows[rows > 0], np.array(grp)
        return rows.max() / rows.min(), grp[grp > 0].max() / grp[grp > 0].min()

    r0, g0 = spreads(np.ones(A.shape[0]), np.ones(A.shape[1]))
    assert r0 > 1.2 or g0 > 1.2
    D, E = block_scalar_equilibration(A, prob.n_free, prob.psd_dims, 300)
    clamped = (D <= 1e-4) | (D >= 1e4)
    assert clamped.sum() <= 0.05 * len(D)      # rows of tiny norm (Lyapunov: 49 of 1134) reach the clamp
    if not clamped.any():
        assert abs(np.mean(np.log(D))) < 1e-12
    r1, g1 = spreads(D, E)
    assert r1 < 1 + 1e-6, r1
    if not clamped.any():
        assert g1 < 1 + 1e-6, g1
    else:                      # clamped rows still weigh in the column norms they touch
        assert g1 < g0, (g0, g1)


def test_scaled_solves_reach_closed_forms():
    r = Oracle.from_problem(F.univariate([0.0, 0.0, 1.0]), scale_iters=10).solve(tol=1e-9, max_iters=20000)
    assert r.status == SOLVED and abs(r.x[0]) < 1e-6
    r = Oracle.from_problem(F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]), scale_iters=10).solve(tol=1e-9,
                                                                                              max_iters=20000)
    assert r.status == SOLVED and abs(r.x[0]) < 1e-6
    X = r.x[1:].reshape(3, 3, order="F")
    assert np.allclose(X, [[1, 0, -1], [0, 0, 0], [-1, 0, 1]], atol=1e-5)
    rng = np.random.default_rng(300)
    a = np.concatenate([rng.standard_normal(6), [1.0]])
    pmin = _brute_univariate(a)
    r = Oracle.from_problem(F.univariate(a), scale_iters=10).solve(tol=1e-8, max_iters=50000)
    assert r.status == SOLVED and abs(r.x[0] - pmin) <= 1e-5 * max(1.0, abs(pmin))
    assert Oracle.from_problem(F.infeasible_pop(), scale_iters=10).solve(tol=1e-6, max_iters=5000).status == \
        PRIMAL_INFEASIBLE
    assert Oracle.from_problem(F.unbounded_pop(), scale_iters=10).solve(tol=1e-6, max_iters=5000).status == \
        DUAL_INFEASIBLE


def _original_residuals(prob, r):
    A = sp.csc_matrix(prob.A)
    rp = np.linalg.norm(A @ r.x - prob.b) / (1 + np.linalg.norm(prob.b))
    rd = np.linalg.norm(A.T @ r.y + r.z - prob.c) / (1 + np.linalg.norm(prob.c))
    return rp, rd


@pytest.mark.parametrize("name", ["c1", "lyap_c5"])
def test_scaled_solution_satisfies_the_original_problem(name):
    prob = CASES[name]()
    r = Oracle.from_problem(prob, scale_iters=10).solve(tol=1e-6, max_iters=20000)
    assert r.status == SOLVED
    rp, rd = _original_residuals(prob, r)
    assert rp <= 1.01e-6 and rd <= 1.01e-6, (rp, rd)
    assert abs(r.pobj - prob.c @ r.x) <= 1e-9 * max(1.0, abs(r.pobj))


class _WrongUnscale(Oracle):
    """Planted mistake: y divided by the row scaling instead of multiplied by it."""
    def unscale(self, u, v):
        n, m = self.n, self.m
        uo, vo = u.copy(), v.copy()
        uo[:n] *= self.E
        uo[n:n + m] /= self.D
        vo[:n] /= self.E
        return uo, vo


def test_planted_unscale_mistake_is_caught():
    prob = CASES["c1"]()
    r = _WrongUnscale.from_problem(prob, scale_iters=10).solve(tol=1e-6, max_iters=20000)
    rp, rd = _original_residuals(prob, r)
    assert r.status != SOLVED or rd > 1e-4


# ---------------------------------------------------------------- weighted SOS vs extra polynomial
def _lowrank_width(prob):
    """Free columns plus lower-triangle PSD columns with two or more nonzeros, counted from A."""
    A = sp.csc_matrix(prob.A)
    nnz = np.diff(A.indptr)
    k = prob.n_free
    off = prob.n_free
    for N in prob.psd_dims:
        for j in range(N):
            for i in range(j, N):
                k += nnz[off + j * N + i] >= 2
        off += N * N
    return int(k)


@pytest.mark.parametrize("n,d", [(3, 2), (3, 3), (2, 3)])
def test_ball_pop_forms_agree_and_auto_takes_the_narrower(n, d):
    w = F.pop_ball(n, 1, form="weighted", half_degree=d)
    e = F.pop_ball(n, 1, form="extra", half_degree=d)
    a = F.pop_ball(n, 1, form="auto", half_degree=d)
    kw, ke = _lowrank_width(w), _lowrank_width(e)
    assert (kw, ke) == (w.meta["k_weighted"], w.meta["k_extra"])      # the widths the choice uses
    assert a.meta["form"] == ("weighted" if kw <= ke else "extra")
    assert e.psd_dims == w.psd_dims and e.m > w.m                     # same Gram blocks, more rows
    gw = Oracle.from_problem(w).solve(tol=1e-8, max_iters=40000)
    ge = Oracle.from_problem(e).solve(tol=1e-8, max_iters=40000)
    assert gw.status == ge.status == SOLVED
    assert abs(gw.x[0] - ge.x[0]) <= 1e-6 * max(1.0, abs(gw.x[0]))   # one relaxation, two encodings


def test_auto_form_choice_at_a_degree_two_multiplier():
    # 2d = 6, n = 3: the multiplier's Gram block has N = 10, weighted width 1 + 55 against 1 + 35
    a = F.pop_ball(3, 0, form="auto", half_degree=3)
    assert a.meta["form"] == "extra" and a.meta["k_weighted"] == 56 and a.meta["k_extra"] == 36
