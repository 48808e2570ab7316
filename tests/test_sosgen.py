"""Generator pins: sizes, partial orthogonality, and the meaning of every row of A.

Nothing here runs the ADMM; these tests fix what the conic data means so that
the oracle and the GPU library are both checked against the paper's model.
"""
import json
import os
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

from sosgen import Poly, families as F, monomials, n_monomials

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table3_example_pop.json")))


def test_basis_order_and_size():
    # graded order 1, x1..xn, x1^2, x1x2, ... (Section I, the candidate monomial vector)
    b = monomials(3, 2)
    assert b[:4] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    assert b[4:7] == [(2, 0, 0), (1, 1, 0), (1, 0, 1)]
    assert b[-1] == (0, 0, 2)
    for n in range(1, 7):
        for d in range(0, 4):
            assert len(monomials(n, d)) == comb(n + d, d) == n_monomials(n, d)


def test_text_sizes_n16_degree6():
    # Section IV-B: 2d = 6, n = 16 gives N = 969 and m = 74 613
    ts = GOLD["text_sizes"]
    N, m = F.shape_counts(ts["n"], ts["two_d"])
    assert (N, m) == (ts["N"], ts["m"])


@pytest.mark.parametrize("n", [10, 12])
def test_table1_dims_from_generator(n):
    # Table I: N = C(n+2,2), m (without the constant moment) = C(n+4,4) - 1, t = C(n+2,2)
    N_t, m_t, t_t = GOLD["table1_dims"][str(n)]
    prob = F.example_pop(n)
    assert max(prob.psd_dims) == N_t
    assert prob.m - 1 == m_t
    assert comb(n + 2, 2) == t_t          # svec size of the (n+1)x(n+1) multiplier Gram block
    assert prob.psd_dims[1] == n + 1


def test_table_dims_closed_forms():
    for n, (N, m, t) in GOLD["table1_dims"].items():
        n = int(n)
        assert (comb(n + 2, 2), comb(n + 4, 4) - 1, comb(n + 2, 2)) == (N, m, t)
    for n, (N, m, t) in GOLD["table2_dims"].items():
        n = int(n)
        assert (comb(n + 2, 2) - 1, comb(n + 4, 4) + n * n - 1, n * (n + 1)) == (N, m, t)


def _indicator_counts(n, d):
    """n_alpha from the polynomial (sum_beta x^beta)^2, i.e. v_d v_d^T summed entrywise."""
    s = Poly(n, {e: 1.0 for e in monomials(n, d)})
    return (s * s).terms


@pytest.mark.parametrize("n,d", [(1, 2), (2, 2), (3, 2), (4, 2), (3, 3)])
def test_partial_orthogonality_prop1(n, d):
    # Proposition 1: A_2 A_2^T = diag(n_alpha), n_alpha = number of nonzeros of B_alpha
    prob = F.pop_from_poly(Poly(n, {(0,) * n: 1.0}), d)
    A2 = prob.A[:, prob.n_free:]
    G = (A2 @ A2.T).toarray()
    assert np.array_equal(G, np.diag(np.diag(G)))
    counts = _indicator_counts(n, d)
    rows = monomials(n, 2 * d)
    assert np.array_equal(np.diag(G), np.array([counts[e] for e in rows]))
    N = comb(n + d, d)
    assert np.diag(G).sum() == N * N
    # and A A^T = D + A_1 A_1^T
    A1 = prob.A[:, :prob.n_free]
    assert np.array_equal((prob.A @ prob.A.T).toarray(), G + (A1 @ A1.T).toarray())


def test_weighted_block_not_orthogonal_but_s0_is():
    # Section VI: the weighted block's indicator matrices overlap; the s0 block's rows stay orthogonal
    prob = F.pop_ball(3, 0)
    N0, N1 = prob.psd_dims
    A0 = prob.A[:, 1:1 + N0 * N0]
    A1 = prob.A[:, 1 + N0 * N0:]
    G0 = (A0 @ A0.T).toarray()
    G1 = (A1 @ A1.T).toarray()
    assert np.array_equal(G0, np.diag(np.diag(G0)))
    assert np.count_nonzero(G1 - np.diag(np.diag(G1))) > 0


def _poly_from_row_coeffs(n, row_degree, coeffs):
    return Poly(n, dict(zip(monomials(n, row_degree), coeffs)))


def test_rows_are_coefficient_matching_pop():
    # For any Gram matrix X, A_2 vec(X) lists the coefficients of v^T X v (Section II-C).
    rng = np.random.default_rng(1)
    n, d = 3, 2
    prob = F.pop_from_poly(Poly(n, {(0,) * n: 1.0}), d)
    N = prob.psd_dims[0]
    R = rng.standard_normal((N, N))
    X = R + R.T
    coeffs = prob.A[:, 1:] @ X.reshape(-1, order="F")
    poly = _poly_from_row_coeffs(n, 2 * d, coeffs)
    basis = monomials(n, d)
    for _ in range(5):
        x = rng.standard_normal(n)
        v = np.array([np.prod(x ** np.array(e)) for e in basis])
        assert abs(poly(x) - v @ X @ v) <= 1e-10 * (1 + abs(v @ X @ v))


def test_rows_are_coefficient_matching_ball():
    # weighted block: row coefficients of q(x) v^T X1 v with q = 1 - |x|^2 (Section VI)
    rng = np.random.default_rng(2)
    n = 2
    prob = F.pop_ball(n, 0)
    N0, N1 = prob.psd_dims
    R = rng.standard_normal((N1, N1))
    X1 = R + R.T
    coeffs = prob.A[:, 1 + N0 * N0:] @ X1.reshape(-1, order="F")
    poly = _poly_from_row_coeffs(n, 4, coeffs)
    basis = monomials(n, 1)
    for _ in range(5):
        x = rng.standard_normal(n)
        v = np.array([np.prod(x ** np.array(e)) for e in basis])
        ref = (1 - x @ x) * (v @ X1 @ v)
        assert abs(poly(x) - ref) <= 1e-10 * (1 + abs(ref))


def test_lyapunov_rows_match_the_two_conditions():
    # s1 = V - eps|x|^2 and s2 = -grad V . f - eps|x|^2, evaluated pointwise (Section II-B)
    n = 2
    rng = np.random.default_rng(3)
    sigma, coef, f = F.lyapunov_field(n, rng)
    prob = F.lyapunov_from_field(n, f, eps=1.0)
    t = prob.n_free
    u = rng.standard_normal(t)
    rhs = prob.b - prob.A[:, :t] @ u            # = coefficients of the two SOS polynomials
    m1 = comb(n + 4, 4)
    s1 = _poly_from_row_coeffs(n, 4, rhs[:m1])
    s2 = _poly_from_row_coeffs(n, 6, rhs[m1:])
    vm = monomials(n, 4, min_degree=2)

    def V(x):
        return sum(ui * np.prod(x ** np.array(e)) for ui, e in zip(u, vm))

    for _ in range(4):
        x = rng.standard_normal(n) * 0.7
        h = 1e-6
        grad = np.array([(V(x + h * np.eye(n)[k]) - V(x - h * np.eye(n)[k])) / (2 * h) for k in range(n)])
        fx = np.array([fi(x) for fi in f])
        assert abs(s1(x) - (V(x) - x @ x)) < 1e-9 * (1 + abs(V(x)))
        ref2 = -grad @ fx - x @ x
        assert abs(s2(x) - ref2) < 1e-5 * (1 + abs(ref2))


def test_family_shapes():
    c1 = F.FAMILIES["c1"](0)
    assert c1.psd_dims == [15] and c1.m == 70 and c1.n_free == 1
    c5 = F.FAMILIES["c5"](0)
    assert c5.psd_dims == [28, 84] and c5.m == 1134 and c5.n_free == 203
    c3 = F.FAMILIES["c3"](0)
    assert c3.psd_dims == [153, 17] and c3.m == 4845
    for s in range(5):
        p = F.pop_batch_member(s)
        n = p.meta["n_vars"]
        assert 6 <= n <= 16 and p.psd_dims == [comb(n + 2, 2)]
    assert F.lyapunov_features(7).shape == (127,)
    assert np.allclose(F.lyapunov_features(7), F.lyapunov(7).meta["features"])


def test_c2_generator_shape_and_law():
    p = F.pop_unconstrained(20, 0, cross_std=0.1)
    assert p.psd_dims == [231] and p.m == 10626
    # b holds p's coefficients; the 8 835 quartic cross terms have std ~0.1, x_i^4 has coefficient 1
    rows = monomials(20, 4)
    quart = np.array([i for i, e in enumerate(rows) if sum(e) == 4 and max(e) < 4])
    assert len(quart) == 8835
    assert 0.09 < np.std(p.b[quart]) < 0.11
    pure = [i for i, e in enumerate(rows) if max(e) == 4]
    assert np.all(p.b[pure] == 1.0)
