"""CPU oracle for solution post-processing of SOS programs (FP64, numpy).

TEST INFRASTRUCTURE.  Only tests/ may import this module (the GPU library and the package
never do); it shares no code with the package's post-processing.

What it computes (Zheng, Fantuzzi, Papachristodoulou, arXiv 1708.04174):

* The SOS decomposition a Gram matrix certifies (Section I, the Gram identity p = v^T X v;
  Section II-C, coefficient matching): X = V diag(lambda) V^T with lambda >= 0 gives
  p(x) - gamma = sum_i q_i(x)^2, q_i = sqrt(lambda_i) v_i^T m(x), m(x) the monomial basis.
* The coefficient residual of that identity: for every monomial x^alpha, the coefficient of
  p - gamma minus that of m(x)^T X m(x), i.e. the sum of X_rs over the pairs of basis monomials
  whose product is x^alpha.
* The moments of the dual of a POP relaxation (max gamma s.t. p - gamma SOS): with cost -1 on
  gamma, the dual variable y of the coefficient rows satisfies -y_0 = 1 and the dual slack of the
  Gram block is the moment matrix sum_alpha (-y_alpha) B_alpha.  When that matrix has rank one,
  the first-order moments (-y at x_1 .. x_n) are the global minimiser.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

Exp = Tuple[int, ...]


def gram_factors(X: np.ndarray):
    """Eigen-decomposition of the symmetrised Gram matrix, eigenvalues clamped at zero,
    largest first: (lambda, V) with X ~= V diag(lambda) V^T."""
    lam, V = np.linalg.eigh(0.5 * (X + X.T))
    order = np.argsort(lam)[::-1]
    return np.maximum(lam[order], 0.0), V[:, order]


def sos_terms(lam: np.ndarray, V: np.ndarray, basis: Sequence[Exp]) -> List[Dict[Exp, float]]:
    """The polynomials q_i = sqrt(lambda_i) v_i^T m(x) (nonzero lambda only), as dicts."""
    out = []
    for i, l in enumerate(lam):
        if l <= 0.0:
            continue
        s = np.sqrt(l)
        out.append({tuple(e): s * V[r, i] for r, e in enumerate(basis) if V[r, i] != 0.0})
    return out


def square_sum(terms: List[Dict[Exp, float]]) -> Dict[Exp, float]:
    """Coefficients of sum_i q_i(x)^2, by multiplying out every product of two terms."""
    acc: Dict[Exp, float] = {}
    for q in terms:
        items = list(q.items())
        for e1, c1 in items:
            for e2, c2 in items:
                e = tuple(a + b for a, b in zip(e1, e2))
                acc[e] = acc.get(e, 0.0) + c1 * c2
    return acc


def identity_residual(p: Dict[Exp, float], gamma: float, sq: Dict[Exp, float], n: int) -> float:
    """max over monomials of |coefficient of (p - gamma) - coefficient of sum_i q_i^2|."""
    target = dict(p)
    zero = (0,) * n
    target[zero] = target.get(zero, 0.0) - gamma
    keys = set(target) | set(sq)
    return max(abs(target.get(e, 0.0) - sq.get(e, 0.0)) for e in keys)


def moments(y: np.ndarray, row_basis: Sequence[Exp]) -> Dict[Exp, float]:
    """Moments m_alpha = -y_alpha of a POP relaxation with cost -gamma, normalised by m_0."""
    m = {tuple(e): -float(v) for e, v in zip(row_basis, y)}
    m0 = m[tuple([0] * len(row_basis[0]))]
    return {e: v / m0 for e, v in m.items()}


def moment_matrix(mom: Dict[Exp, float], basis: Sequence[Exp]) -> np.ndarray:
    """M[r][s] = m at the product of basis monomials r and s."""
    N = len(basis)
    M = np.empty((N, N))
    for r in range(N):
        for s in range(N):
            M[r, s] = mom[tuple(a + b for a, b in zip(basis[r], basis[s]))]
    return M


def extract_minimiser(mom: Dict[Exp, float], basis: Sequence[Exp], n: int):
    """(x*, rank-one ratio): x*_i = m at x_i; the ratio of the moment matrix's second to first
    eigenvalue (small when the relaxation's optimum is a single point, then x* is it)."""
    x = np.array([mom[tuple(1 if j == i else 0 for j in range(n))] for i in range(n)])
    w = np.linalg.eigvalsh(moment_matrix(mom, basis))
    return x, float(w[-2] / w[-1]) if len(w) > 1 else 0.0


def evaluate(p: Dict[Exp, float], x: np.ndarray) -> float:
    return float(sum(c * np.prod(np.asarray(x, dtype=float) ** np.array(e)) for e, c in p.items()))
