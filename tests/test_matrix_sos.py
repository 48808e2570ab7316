"""Matrix-valued SOS programs (Section V): the coefficient-matching structure of Proposition 2,
and the oracle's optimal values against brute force (univariate matrix polynomials that are PSD
for every x are SOS matrices, so max gamma s.t. P - gamma I SOS equals min_x lambda_min(P(x)))."""
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import minimize_scalar

from oracle.admm import SOLVED, Oracle
from sosgen import matrix_sos as M


def _min_eig_univariate(P):
    f = lambda x: np.linalg.eigvalsh(M.evaluate(P, [x]))[0]
    g = np.linspace(-6, 6, 12001)
    v = np.array([f(x) for x in g])
    x0 = g[np.argmin(v)]
    return minimize_scalar(f, bracket=(x0 - 0.002, x0, x0 + 0.002)).fun


@pytest.mark.parametrize("n,r", [(1, 2), (2, 3), (3, 2)])
def test_structure_is_partially_orthogonal(n, r):
    prob = M.matrix_pop(n, r, 0)
    N = comb(n + 2, 2)
    L = r * N
    assert prob.psd_dims == [L] and prob.m == r * (r + 1) // 2 * comb(n + 4, 4)
    A = sp.csc_matrix(prob.A)
    nnz = np.diff(A.indptr)[prob.n_free:]
    assert np.all(nnz == 1)                                      # every entry of Y in one row
    Y = A[:, prob.n_free:]
    perm = np.arange(L * L).reshape(L, L).T.reshape(-1)
    assert abs(Y - Y[:, perm]).sum() == 0.0                      # columns (p,q) and (q,p) identical
    G = (Y @ Y.T).toarray()
    assert np.allclose(G, np.diag(np.diag(G)), atol=0.0)         # A_s A_s^T diagonal (Proposition 2)


@pytest.mark.parametrize("r,seed", [(2, 0), (3, 1), (2, 5)])
def test_univariate_matrix_bound_equals_min_eigenvalue(r, seed):
    prob = M.matrix_pop(1, r, seed)
    ref = _min_eig_univariate(prob.meta["P"])
    res = Oracle.from_problem(prob).solve(tol=1e-9, max_iters=80000)
    assert res.status == SOLVED
    assert abs(res.x[0] - ref) <= 1e-5 * max(1.0, abs(ref)), (res.x[0], ref)


def test_block_diagonal_matrix_decouples():
    # P = diag(p1, p2) with univariate quartics: gamma* = min(min p1, min p2)
    p1 = np.array([0.3, -1.0, 0.2, 0.5, 1.0])
    p2 = np.array([-0.7, 0.4, -1.5, -0.2, 1.0])
    P = {(k,): np.diag([p1[k], p2[k]]) for k in range(5)}
    prob = M.build_matrix_sos_sdp(1, 2, 2, P, [{(0,): np.eye(2)}], [-1.0])
    ref = min(min(np.polyval(a[::-1], c.real) for c in np.roots(np.polyder(a[::-1])) if abs(c.imag) < 1e-9)
              for a in (p1, p2))
    res = Oracle.from_problem(prob).solve(tol=1e-9, max_iters=80000)
    assert res.status == SOLVED and abs(res.x[0] - ref) <= 1e-5 * max(1.0, abs(ref))


def test_multivariate_bound_is_below_sampled_minimum():
    prob = M.matrix_pop(2, 3, 2)
    res = Oracle.from_problem(prob).solve(tol=1e-7, max_iters=40000)
    assert res.status == SOLVED
    rng = np.random.default_rng(1)
    sampled = min(np.linalg.eigvalsh(M.evaluate(prob.meta["P"], rng.uniform(-3, 3, 2)))[0] for _ in range(4000))
    assert res.x[0] <= sampled + 1e-6 and res.x[0] >= sampled - 0.05 * abs(sampled)


def test_planted_off_diagonal_factor_mistake_is_caught():
    # dropping the factor 2 of the i < j rows' right-hand side matches half the off-diagonal part
    prob = M.matrix_pop(1, 2, 0)
    ref = _min_eig_univariate(prob.meta["P"])
    b = prob.b.copy()
    ma = 5
    b[ma:2 * ma] *= 0.5          # rows of the pair (0, 1)
    res = Oracle(prob.A, b, prob.c, prob.n_free, prob.psd_dims).solve(tol=1e-9, max_iters=80000)
    assert abs(res.x[0] - ref) > 1e-3
