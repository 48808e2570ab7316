"""CPU FP64 oracle: HSDE-ADMM on an SOS-derived SDP, with I + A A^T factored directly.

TEST INFRASTRUCTURE.  Only tests/, the smoke check in __graft_entry__.py and the
cpu_baseline leg of bench.py may import or run anything in oracle/.  The GPU
library never calls it, and the two share no code: the only common input is the
conic data (A, b, c, K) produced by the seeded generators in sosgen/.

What it computes (Zheng, Fantuzzi, Papachristodoulou, arXiv 1708.04174):

* The conic program min c^T xi s.t. A xi = b, xi in K (Section III) and its dual
  max b^T y s.t. A^T y + z = c, z in K* (Section IV-A), embedded in the
  homogeneous self-dual system v = Q u with u = (xi, y, tau), v = (z, s, kappa)
  and the skew matrix Q of Section IV-A.
* The three ADMM steps of Section IV-A: an affine solve with I + Q, a projection
  onto C = K x R^m x R_+, and the dual update.
* The affine solve is written out the way Section IV-B eliminates it: u3 is
  eliminated (the system with M + zeta zeta^T), the rank-one term is removed with
  the matrix inversion lemma using the cached h = M^{-1} zeta, and the M-system is
  reduced to (I + A A^T) sigma_2 = w2 - A w1, sigma_1 = w1 + A^T sigma_2.
  Here I + A A^T is factored DIRECTLY (dense Cholesky for m <= 8000, otherwise a
  sparse LU of the explicit matrix) - the partial-orthogonality trick of
  Section IV-B is deliberately NOT used, so the GPU path that does use it is
  checked against an independent route to the same iterates.
* The PSD projection uses LAPACK eigh on the symmetrised block, clamps the
  eigenvalues at zero and rebuilds V max(L, 0) V^T.

Readings where the paper is silent:
* start point u = v = (0, 0, 1), as in the ADMM paper the method builds on;
* relaxation alpha = 1 (the paper's three steps have none);
* stopping: max(r_p, r_d, r_g) <= tol with the normalised residuals below,
  infeasibility from the embedding's certificates (tau -> 0, kappa > 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

SOLVED = 1
PRIMAL_INFEASIBLE = 2
DUAL_INFEASIBLE = 3
MAX_ITERS = 4
STATUS_NAMES = {SOLVED: "solved", PRIMAL_INFEASIBLE: "primal_infeasible",
                DUAL_INFEASIBLE: "dual_infeasible", MAX_ITERS: "max_iters"}


def validate(A, b, c, n_free: int, psd_dims: List[int]) -> None:
    """Shapes, finiteness, and symmetric column pairs (i,j)/(j,i) inside every PSD block."""
    m, n = A.shape
    if n != n_free + sum(N * N for N in psd_dims):
        raise ValueError("A has the wrong number of columns for the cone")
    if b.shape != (m,) or c.shape != (n,):
        raise ValueError("b or c has the wrong length")
    if not (np.all(np.isfinite(A.data)) and np.all(np.isfinite(b)) and np.all(np.isfinite(c))):
        raise ValueError("non-finite data")
    A = sp.csc_matrix(A)
    off = n_free
    for N in psd_dims:
        blk = A[:, off:off + N * N]
        perm = np.arange(N * N).reshape(N, N).T.reshape(-1)    # column (i,j) <-> (j,i)
        if abs(blk - blk[:, perm]).sum() != 0.0:
            raise ValueError("PSD block columns are not symmetric")
        cb = c[off:off + N * N]
        if np.any(cb != cb[perm]):
            raise ValueError("cost on a PSD block is not symmetric")
        off += N * N


def block_scalar_equilibration(A, n_free: int, psd_dims: List[int], iters: int):
    """Row scaling D (m) and column scaling E (n) with E constant on every PSD block.

    Ruiz's alternating equilibration (rows and columns divided by the square roots of their
    norms, repeated), restricted so that the scaled matrix D A E keeps partial orthogonality:
    a diagonal D keeps A_s A_s^T diagonal (D A_s A_s^T D), and one factor e per PSD block keeps
    the block's columns, hence the cone, intact (A_s e^2 A_s^T).  Norms are 2-norms over the
    full-vec columns; a PSD block's factor uses the root mean square of its N^2 column norms;
    each free variable is its own group.  D A E does not fix how the scaling splits between D
    and E ((s D, E / s) gives the same matrix but shifts the weight between primal and dual
    residuals), and with m != n the passes drift in s, so after every pass D is divided by its
    geometric mean and E multiplied by it: the row scaling stays neutral on average.  Then the
    factors are clamped to [1e-4, 1e4].  Rows and column groups cannot all reach norm 1 unless
    m equals n (both conditions fix the Frobenius norm of D A E); the passes drive every row
    to one common norm and every group to another."""
    A = sp.csc_matrix(A, dtype=np.float64)
    m, n = A.shape
    D = np.ones(m)
    E = np.ones(n)
    groups = [(j, j + 1) for j in range(n_free)]
    off = n_free
    for N in psd_dims:
        groups.append((off, off + N * N))
        off += N * N
    A2 = A.multiply(A).tocsc()     # squared entries
    for _ in range(iters):
        r = np.sqrt(np.asarray((A2 @ (E * E))).ravel()) * D        # |row_i of D A E|
        D = D / np.sqrt(np.where(r > 0, r, 1.0))
        cn2 = np.asarray(A2.T @ (D * D)).ravel() * E * E            # |col_j of D A E|^2
        for a, b in groups:
            val = np.sqrt(cn2[a:b].mean())
            if val > 0:
                E[a:b] = E[a:b] / np.sqrt(val)
        g = np.exp(np.mean(np.log(D)))
        D = np.clip(D / g, 1e-4, 1e4)
        E = np.clip(E * g, 1e-4, 1e4)
    return D, E


def proj_psd(W: np.ndarray) -> np.ndarray:
    """Euclidean projection of a symmetric matrix onto S_+: V max(lambda, 0) V^T."""
    S = 0.5 * (W + W.T)
    lam, V = np.linalg.eigh(S)
    return (V * np.maximum(lam, 0.0)) @ V.T


@dataclass
class OracleResult:
    status: int
    iters: int
    pobj: float
    dobj: float
    res_pri: float
    res_dual: float
    gap: float
    tau: float
    kappa: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    u: np.ndarray
    v: np.ndarray
    gamma: Optional[float] = None
    history: list = field(default_factory=list)

    @property
    def status_name(self) -> str:
        return STATUS_NAMES[self.status]


class Oracle:
    """Plain FP64 HSDE-ADMM for min c^T xi, A xi = b, xi in R^{n_free} x S^{N_1}_+ x ... (full vec)."""

    def __init__(self, A, b, c, n_free: int, psd_dims: List[int], dense_limit: int = 8000, scale_iters: int = 0):
        """scale_iters > 0: iterate on the equilibrated problem D A E, D b, E c
        (block_scalar_equilibration); iterates, residuals and certificates are reported in the
        original units, x = E x^, y = D y^, z = z^ / E."""
        A = sp.csc_matrix(A, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        c = np.asarray(c, dtype=np.float64)
        validate(A, b, c, n_free, list(psd_dims))
        self.A0, self.A0t = A, sp.csr_matrix(A.T)   # original data: residuals are taken in its units
        self.b0, self.c0 = b, c
        if scale_iters > 0:
            self.D, self.E = block_scalar_equilibration(A, n_free, list(psd_dims), scale_iters)
            A = sp.csc_matrix(sp.diags(self.D) @ A @ sp.diags(self.E))
            b, c = self.D * b, self.E * c
        else:
            self.D, self.E = np.ones(A.shape[0]), np.ones(A.shape[1])
        self.A, self.At = A, sp.csr_matrix(A.T)
        self.b, self.c = b, c
        self.m, self.n = A.shape
        self.n_free = n_free
        self.psd_dims = list(psd_dims)
        # I + A A^T, factored directly (no diagonal-plus-low-rank split)
        F = (sp.identity(self.m, format="csc") + (A @ A.T).tocsc()).tocsc()
        if self.m <= dense_limit:
            self._chol = sla.cho_factor(F.toarray(), lower=True)
            self._lu = None
        else:
            self._chol = None
            self._lu = spla.splu(F)
        # h = M^{-1} zeta with zeta = (c, -b), and 1 + zeta^T h  (Section IV-B, rank-one term)
        h1, h2 = self.solve_M(c, -b)
        self.h = np.concatenate([h1, h2])
        self.eta = 1.0 + c @ h1 - b @ h2

    @classmethod
    def from_problem(cls, prob, **kw) -> "Oracle":
        return cls(prob.A, prob.b, prob.c, prob.n_free, prob.psd_dims, **kw)

    # ------------------------------------------------------------ linear algebra
    def solve_F(self, r: np.ndarray) -> np.ndarray:
        """(I + A A^T)^{-1} r."""
        if self._chol is not None:
            return sla.cho_solve(self._chol, r)
        return self._lu.solve(r)

    def solve_M(self, w1: np.ndarray, w2: np.ndarray):
        """Solve [I -A^T; A I][s1; s2] = [w1; w2] by eliminating s1 (Section IV-B)."""
        s2 = self.solve_F(w2 - self.A @ w1)
        s1 = w1 + self.At @ s2
        return s1, s2

    def affine(self, omega: np.ndarray) -> np.ndarray:
        """u_hat = (I + Q)^{-1} omega for omega = (w1, w2, w3)."""
        n, m = self.n, self.m
        w1, w2, w3 = omega[:n], omega[n:n + m], omega[n + m]
        # right-hand side of (M + zeta zeta^T)[u1; u2] = [w1; w2] - w3 zeta
        s1, s2 = self.solve_M(w1 - self.c * w3, w2 + self.b * w3)
        # matrix inversion lemma for the rank-one zeta zeta^T
        theta = (self.c @ s1 - self.b @ s2) / self.eta
        u1 = s1 - theta * self.h[:n]
        u2 = s2 - theta * self.h[n:]
        # back-substitution for the eliminated third block
        u3 = w3 + self.c @ u1 - self.b @ u2
        return np.concatenate([u1, u2, [u3]])

    def Q_matvec(self, u: np.ndarray) -> np.ndarray:
        """Q u with Q = [[0, -A^T, c], [A, 0, -b], [-c^T, b^T, 0]]."""
        n, m = self.n, self.m
        x, y, t = u[:n], u[n:n + m], u[n + m]
        return np.concatenate([-(self.At @ y) + self.c * t, self.A @ x - self.b * t,
                               [-(self.c @ x) + self.b @ y]])

    # ------------------------------------------------------------ cone projection
    def project_K(self, x: np.ndarray) -> np.ndarray:
        out = x.copy()
        off = self.n_free
        for N in self.psd_dims:
            W = x[off:off + N * N].reshape(N, N, order="F")
            out[off:off + N * N] = proj_psd(W).reshape(-1, order="F")
            off += N * N
        return out

    def project_C(self, w: np.ndarray) -> np.ndarray:
        """Projection onto C = K x R^m x R_+."""
        n = self.n
        out = w.copy()
        out[:n] = self.project_K(w[:n])
        out[-1] = max(w[-1], 0.0)
        return out

    # ------------------------------------------------------------ iteration
    def initial(self):
        N = self.n + self.m + 1
        u = np.zeros(N)
        v = np.zeros(N)
        u[-1] = 1.0
        v[-1] = 1.0
        return u, v

    def step(self, u: np.ndarray, v: np.ndarray, alpha: float = 1.0):
        """One ADMM iteration (Section IV-A): affine solve, cone projection, dual update."""
        u_hat = self.affine(u + v)
        if alpha != 1.0:
            u_hat = alpha * u_hat + (1.0 - alpha) * u
        u_new = self.project_C(u_hat - v)
        v_new = v - u_hat + u_new
        return u_new, v_new

    def run(self, iters: int, u=None, v=None, alpha: float = 1.0):
        if u is None:
            u, v = self.initial()
        for _ in range(iters):
            u, v = self.step(u, v, alpha)
        return u, v

    # ------------------------------------------------------------ termination
    def unscale(self, u: np.ndarray, v: np.ndarray):
        """Iterate of the equilibrated problem -> the same iterate in the original units."""
        n, m = self.n, self.m
        uo, vo = u.copy(), v.copy()
        uo[:n] *= self.E
        uo[n:n + m] *= self.D
        vo[:n] /= self.E
        return uo, vo

    def rescale(self, u: np.ndarray, v: np.ndarray):
        """Inverse of unscale."""
        n, m = self.n, self.m
        ui, vi = u.copy(), v.copy()
        ui[:n] /= self.E
        ui[n:n + m] /= self.D
        vi[:n] *= self.E
        return ui, vi

    def residuals(self, u: np.ndarray, v: np.ndarray) -> dict:
        """Residuals and certificate tests in the original units (for an equilibrated problem,
        of the unscaled iterate: A x - b tau = D^-1 (A^ x^ - b^ tau), and so on)."""
        n, m = self.n, self.m
        u, v = self.unscale(u, v)
        xi, y, tau = u[:n], u[n:n + m], u[n + m]
        z, kappa = v[:n], v[n + m]
        b0, c0 = self.b0, self.c0
        nb = np.linalg.norm(b0)
        nc = np.linalg.norm(c0)
        Ax = self.A0 @ xi
        Aty = self.A0t @ y
        cx = c0 @ xi
        by = b0 @ y
        out = {"tau": tau, "kappa": kappa, "cx": cx, "by": by}
        if tau > 0.0:
            out["res_pri"] = np.linalg.norm(Ax - b0 * tau) / tau / (1.0 + nb)
            out["res_dual"] = np.linalg.norm(Aty + z - c0 * tau) / tau / (1.0 + nc)
            out["gap"] = abs(cx - by) / tau / (1.0 + abs(cx) / tau + abs(by) / tau)
            out["pobj"] = cx / tau
            out["dobj"] = by / tau
        else:
            out.update(res_pri=np.inf, res_dual=np.inf, gap=np.inf, pobj=np.nan, dobj=np.nan)
        out["pinf"] = np.linalg.norm(Aty + z)     # primal infeasibility certificate test
        out["dinf"] = np.linalg.norm(Ax)          # dual infeasibility certificate test
        return out

    def status_of(self, r: dict, tol: float) -> int:
        if max(r["res_pri"], r["res_dual"], r["gap"]) <= tol:
            return SOLVED
        if r["by"] > 0.0 and r["pinf"] <= tol * r["by"]:
            return PRIMAL_INFEASIBLE
        if r["cx"] < 0.0 and r["dinf"] <= tol * (-r["cx"]):
            return DUAL_INFEASIBLE
        return 0

    def solve(self, tol: float = 1e-4, max_iters: int = 2000, check_every: int = 10,
              alpha: float = 1.0, u=None, v=None, keep_history: bool = False) -> OracleResult:
        if u is None:
            u, v = self.initial()
        status, it, hist = MAX_ITERS, 0, []
        r = None
        for it in range(1, max_iters + 1):
            u, v = self.step(u, v, alpha)
            if it % check_every == 0 or it == max_iters:
                r = self.residuals(u, v)
                if keep_history:
                    hist.append((it, r["res_pri"], r["res_dual"], r["gap"]))
                s = self.status_of(r, tol)
                if s:
                    status = s
                    break
        if r is None:
            r = self.residuals(u, v)
        n, m = self.n, self.m
        u, v = self.unscale(u, v)
        tau = u[n + m]
        scale = 1.0 / tau if tau > 0 else 1.0
        res = OracleResult(status=status, iters=it, pobj=r["pobj"], dobj=r["dobj"], res_pri=r["res_pri"],
                           res_dual=r["res_dual"], gap=r["gap"], tau=tau, kappa=v[n + m],
                           x=u[:n] * scale, y=u[n:n + m] * scale, z=v[:n] * scale, u=u, v=v, history=hist)
        return res


def gamma_of(result: OracleResult, gamma_index: int = 0) -> float:
    """For max gamma programs written with cost -gamma: gamma = xi[gamma_index] (already divided by tau)."""
    return float(result.x[gamma_index])
