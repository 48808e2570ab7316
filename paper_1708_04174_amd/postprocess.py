"""Post-processing of a solved SOS program: the SOS decomposition its Gram matrix certifies,
the coefficient residual of that identity, and the minimiser read off the dual moments.

The eigen-decompositions run in the library (sos_psd_factor, FP64 Jacobi on the device);
this module only indexes monomials.  Facts used (Zheng, Fantuzzi, Papachristodoulou, arXiv
1708.04174, Section I and Section II-C):

* X = sum_j lambda_j v_j v_j^T with lambda_j >= 0 gives p - gamma = sum_j q_j^2 with
  q_j = sqrt(lambda_j) v_j^T m(x), m(x) the Gram block's monomial basis.
* The coefficient of x^alpha in m(x)^T X m(x) is the sum of X_rs over the basis pairs (r, s)
  with product x^alpha; its difference from p - gamma is the identity's residual.
* For max gamma s.t. p - gamma SOS with cost -1 on gamma, -y is the moment vector (-y_0 = 1)
  and the Gram block of Z is its moment matrix; when that matrix has rank one the first-order
  moments are the global minimiser.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import binding as B


@dataclass
class SOSDecomposition:
    gamma: float
    weights: np.ndarray          # lambda_j (clamped at 0), largest first
    vectors: np.ndarray          # N x r: coefficient vectors v_j of q_j / sqrt(lambda_j) over the basis
    basis: List[tuple]           # the block's monomials (exponent tuples)
    residual: float              # max_alpha |coefficient of p - gamma - sum_j q_j^2|


def _row_index(row_basis: Sequence[tuple]):
    return {tuple(e): k for k, e in enumerate(row_basis)}


def sos_decomposition(work, b: np.ndarray, row_basis: Sequence[tuple], basis: Sequence[tuple], block: int = 0,
                      gamma_index: int = 0, rank_tol: float = 0.0) -> SOSDecomposition:
    """Decomposition of the solution's Gram block `block` (its basis `basis`), with p's
    coefficients b over row_basis (coefficient matching puts p_alpha in b_alpha)."""
    lam, V = B.sos_psd_factor(work, block, dual=False)
    order = np.argsort(lam)[::-1]
    lam, V = np.maximum(lam[order], 0.0), V[:, order]
    keep = lam > rank_tol * (lam[0] if len(lam) else 0.0)
    lam, V = lam[keep], V[:, keep]
    x, _, _ = B.sos_get_solution(work)
    gamma = float(x[gamma_index])
    # coefficients of m^T (V diag(lam) V^T) m on the row basis: X_rs accumulated at row(e_r + e_s)
    Xr = (V * lam) @ V.T
    rows = _row_index(row_basis)
    ex = np.array(basis, dtype=np.int64)
    pair = ex[:, None, :] + ex[None, :, :]
    idx = np.array([rows[tuple(e)] for e in pair.reshape(-1, ex.shape[1])]).reshape(len(basis), len(basis))
    coef = np.zeros(len(row_basis))
    np.add.at(coef, idx, Xr)
    target = np.array(b, dtype=float).copy()
    target[rows[(0,) * ex.shape[1]]] -= gamma
    return SOSDecomposition(gamma, lam, V, [tuple(e) for e in basis], float(np.max(np.abs(target - coef))))


def minimiser(work, row_basis: Sequence[tuple], n: int, block: int = 0):
    """(x*, ratio): first-order moments of the dual of a POP relaxation, and the moment matrix's
    second-to-first eigenvalue ratio (small: the moments are those of one point, x* is it)."""
    _, y, _ = B.sos_get_solution(work)
    rows = _row_index(row_basis)
    m0 = -y[rows[(0,) * n]]
    x = np.array([-y[rows[tuple(1 if j == i else 0 for j in range(n))]] / m0 for i in range(n)])
    lam, _ = B.sos_psd_factor(work, block, dual=True)
    lam = np.sort(lam)[::-1]
    return x, float(lam[1] / lam[0]) if len(lam) > 1 else 0.0
