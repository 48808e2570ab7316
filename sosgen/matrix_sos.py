"""Matrix-valued SOS programs (Section V): coefficient matching for

    P_0(x) - sum_h u_h P_h(x) = (I_r (x) v_d(x))^T Y (I_r (x) v_d(x)),   Y in S^{r N}_+,

with P_h symmetric r x r polynomial matrices of degree <= 2d and N = C(n + d, d).  Entry (i, j)
of the right-hand side is sum over basis pairs (a, b) of v_a v_b Y[(i,a),(j,b)], so matching the
coefficient of x^alpha in entry (i, j) gives one row per (alpha, i <= j):

    i = j:  sum_{(a,b): v_a v_b = x^alpha} Y[(i,a),(i,b)]                        = (C_alpha)_ii
    i < j:  sum_{(a,b): v_a v_b = x^alpha} (Y[(i,a),(j,b)] + Y[(j,a),(i,b)])   = 2 (C_alpha)_ij

(the (j,i) equation is the same one for symmetric Y, and writing both halves keeps the columns of
Y's entries (p,q) and (q,p) identical).  Every entry of Y appears in exactly one row, so the Y
columns are mutually orthogonal and A_s A_s^T is diagonal (Proposition 2); the free variables u
form A_f.  Column layout as in Section III: u, then the column-stacked vec of Y.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .poly import monomials
from .sdp import ConicProblem

MatPoly = Dict[Tuple[int, ...], np.ndarray]   # exponent -> symmetric r x r coefficient


def build_matrix_sos_sdp(n: int, half_degree: int, r: int, P0: MatPoly, Ph: Sequence[MatPoly],
                         w: Sequence[float], meta: Optional[dict] = None) -> ConicProblem:
    row_basis = monomials(n, 2 * half_degree)
    row_of = {e: k for k, e in enumerate(row_basis)}
    ma = len(row_basis)
    pairs = [(i, j) for i in range(r) for j in range(i, r)]
    pair_of = {p: k for k, p in enumerate(pairs)}
    basis = np.array(monomials(n, half_degree), dtype=np.int64).reshape(-1, n)
    N = basis.shape[0]
    L = r * N
    t = len(Ph)
    m = len(pairs) * ma

    def row(alpha, i, j):
        return pair_of[(i, j)] * ma + row_of[tuple(alpha)]

    def mult(i, j):
        return 1.0 if i == j else 2.0

    b = np.zeros(m)
    for e, C in P0.items():
        for (i, j) in pairs:
            b[row(e, i, j)] += mult(i, j) * C[i, j]
    rows, cols, vals = [], [], []
    for h, Pm in enumerate(Ph):
        for e, C in Pm.items():
            for (i, j) in pairs:
                if C[i, j] != 0.0:
                    rows.append(row(e, i, j))
                    cols.append(h)
                    vals.append(mult(i, j) * C[i, j])
    # entry (p, q) of Y, p = (i, a), q = (j, b): row (alpha = v_a v_b, min(i,j), max(i,j)), value 1
    for i in range(r):
        for j in range(r):
            lo, hi = min(i, j), max(i, j)
            for a in range(N):
                for bb in range(N):
                    alpha = tuple(basis[a] + basis[bb])
                    p, q = i * N + a, j * N + bb
                    rows.append(row(alpha, lo, hi))
                    cols.append(t + q * L + p)      # column-stacked vec: column q, row p
                    vals.append(1.0)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(m, t + L * L)).tocsc()
    A.sum_duplicates()
    A.sort_indices()
    c = np.zeros(t + L * L)
    c[:t] = np.asarray(w, dtype=float)
    md = {"kind": "matrix_sos", "n_vars": n, "half_degree": half_degree, "r": r, "basis_size": N}
    md.update(meta or {})
    return ConicProblem(A=A, b=b, c=c, n_free=t, psd_dims=[L], meta=md)


def random_matrix_poly(n: int, half_degree: int, r: int, rng: np.random.Generator, lead: float = 1.0) -> MatPoly:
    """Symmetric r x r matrix polynomial: N(0,1) symmetric coefficients on every monomial of degree
    < 2d, and lead * I_r on every x_i^{2d} (so that P(x) - gamma I is PSD for gamma low enough)."""
    P: MatPoly = {}
    for e in monomials(n, 2 * half_degree - 1):
        G = rng.standard_normal((r, r))
        P[tuple(e)] = 0.5 * (G + G.T)
    for i in range(n):
        e = [0] * n
        e[i] = 2 * half_degree
        P[tuple(e)] = P.get(tuple(e), np.zeros((r, r))) + lead * np.eye(r)
    return P


def matrix_pop(n: int, r: int, seed: int, half_degree: int = 2) -> ConicProblem:
    """max gamma s.t. P(x) - gamma I_r is an SOS matrix, P random (random_matrix_poly); cost -gamma."""
    rng = np.random.default_rng(seed)
    P = random_matrix_poly(n, half_degree, r, rng)
    zero = tuple([0] * n)
    return build_matrix_sos_sdp(n, half_degree, r, P, [{zero: np.eye(r)}], [-1.0],
                                {"family": "matrix_pop", "seed": seed, "gamma_index": 0, "P": P})


def evaluate(P: MatPoly, x: Sequence[float]) -> np.ndarray:
    x = np.asarray(x, dtype=float)
    out = None
    for e, C in P.items():
        term = C * float(np.prod(x ** np.array(e)))
        out = term if out is None else out + term
    return out
