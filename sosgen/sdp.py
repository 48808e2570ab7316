"""Coefficient matching: SOS program -> conic data (A, b, c, K).

An SOS program in the paper's standard form (Section II-B, the multi-constraint
program; Section VI for weighted constraints) has t free decision variables u
with cost w, and a list of polynomial identities

    g_0(x) - sum_i u_i g_i(x) = sum_b q_b(x) * v_{d_b}(x)^T X_b v_{d_b}(x),

one per equation, where every X_b is a PSD Gram matrix and q_b is a fixed weight
polynomial (q_b = 1 for a plain SOS polynomial).  Matching the coefficient of
every monomial x^alpha of degree <= 2d on both sides (Section II-C, the
coefficient matching conditions) gives one equality row per alpha:

    <B^{(b)}_alpha, X_b> summed over blocks  +  sum_i u_i g_{i,alpha}  =  g_{0,alpha},

with B_alpha the 0/1 indicator of v v^T (Section II-C) and, for weighted blocks,
B^{(b)}_alpha the indicator of q_b v v^T (Section VI).  The columns are laid out
as in Section III: first the t free variables (A_1, c = [w; 0]), then each PSD
block as the column-stacked vec of its N_b x N_b Gram matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

from .poly import Poly, monomials


@dataclass
class SOSEquation:
    """One polynomial identity g0 - sum_i u_i g[i] = sum_b weight_b * (Gram form of degree 2*half_deg_b).

    Rows are the monomials of degree row_min_degree..row_degree; a block is (half_degree, weight)
    with the Gram basis of all monomials of degree <= half_degree, or (half_degree, weight,
    min_degree) with the basis of degrees min_degree..half_degree (e.g. a form without constant
    or linear terms, as in the local Lyapunov conditions)."""
    row_degree: int                    # rows = monomials of degree <= row_degree
    g0: Poly
    g: Dict[int, Poly]                 # free-variable index -> polynomial g_i (sparse over i)
    blocks: List[tuple]                # (half_degree, weight Poly[, min_degree]) per Gram block
    row_min_degree: int = 0


@dataclass
class ConicProblem:
    """min c^T xi  s.t.  A xi = b,  xi in R^{n_free} x S^{N_1}_+ x ... (full column-stacked vec)."""
    A: sp.csc_matrix
    b: np.ndarray
    c: np.ndarray
    n_free: int
    psd_dims: List[int]
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    def block_offsets(self) -> List[int]:
        offs, o = [], self.n_free
        for N in self.psd_dims:
            offs.append(o)
            o += N * N
        return offs

    def shape_summary(self) -> dict:
        return {"m": self.m, "n": self.n, "n_free": self.n_free, "psd_dims": list(self.psd_dims),
                "nnz": int(self.A.nnz)}


def build_sos_sdp(n: int, n_free: int, w: Sequence[float], equations: Sequence[SOSEquation],
                  meta: Optional[dict] = None) -> ConicProblem:
    """Assemble (A, b, c, K) for the SOS program described by `equations`."""
    rows_i: List[np.ndarray] = []
    cols_i: List[np.ndarray] = []
    vals: List[np.ndarray] = []
    b_parts: List[np.ndarray] = []
    psd_dims: List[int] = []

    # column offsets: free variables first, then every block of every equation
    col = n_free
    block_cols = []
    for eq in equations:
        offs = []
        for blk in eq.blocks:
            N = len(monomials(n, blk[0], blk[2] if len(blk) > 2 else 0))
            offs.append(col)
            psd_dims.append(N)
            col += N * N
        block_cols.append(offs)
    n_cols = col

    row0 = 0
    for eq, offs in zip(equations, block_cols):
        row_basis = monomials(n, eq.row_degree, eq.row_min_degree)
        row_of = {e: k for k, e in enumerate(row_basis)}
        m_eq = len(row_basis)

        def row_index(e) -> int:
            r = row_of.get(tuple(e))
            if r is None:
                raise ValueError(f"monomial {e} is outside the row degrees {eq.row_min_degree}..{eq.row_degree}")
            return r

        # right-hand side b_alpha = g_{0,alpha}
        b_eq = np.zeros(m_eq)
        for e, cf in eq.g0.items():
            b_eq[row_index(e)] += cf
        b_parts.append(b_eq)

        # free-variable columns A_1: entry g_{i,alpha}
        for i, gi in eq.g.items():
            if not 0 <= i < n_free:
                raise ValueError("free-variable index out of range")
            for e, cf in gi.items():
                rows_i.append(np.array([row0 + row_index(e)]))
                cols_i.append(np.array([i]))
                vals.append(np.array([cf]))

        # Gram blocks: entry (r, s) of X_b meets monomial v_r + v_s + delta of the weight
        for blk, off in zip(eq.blocks, offs):
            half_deg, wt = blk[0], blk[1]
            basis = np.array(monomials(n, half_deg, blk[2] if len(blk) > 2 else 0), dtype=np.int64).reshape(-1, n)
            N = basis.shape[0]
            pair = basis[:, None, :] + basis[None, :, :]          # (N, N, n): exponent of v_r v_s
            rr, ss = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
            vec_col = off + ss * N + rr                           # column-stacked vec index of (r, s)
            for de, cf in wt.items():
                ex = pair + np.array(de, dtype=np.int64)
                flat = ex.reshape(-1, n)
                ridx = np.fromiter((row_index(tuple(v)) for v in flat), dtype=np.int64, count=flat.shape[0])
                rows_i.append(row0 + ridx)
                cols_i.append(vec_col.reshape(-1))
                vals.append(np.full(flat.shape[0], cf))
        row0 += m_eq

    r = np.concatenate(rows_i) if rows_i else np.zeros(0, np.int64)
    cidx = np.concatenate(cols_i) if cols_i else np.zeros(0, np.int64)
    v = np.concatenate(vals) if vals else np.zeros(0)
    A = sp.coo_matrix((v, (r, cidx)), shape=(row0, n_cols)).tocsc()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    c = np.zeros(n_cols)
    c[:n_free] = np.asarray(w, dtype=float)
    return ConicProblem(A=A, b=np.concatenate(b_parts), c=c, n_free=n_free,
                        psd_dims=psd_dims, meta=dict(meta or {}))
