"""Seeded problem families shaped like the paper's workloads.

Every generator draws from numpy.random.default_rng(seed) (PCG64), coefficients
in graded monomial order, and returns a ConicProblem.

* pop_unconstrained  - max gamma s.t. p - gamma SOS (Section II-B, the POP relaxation).
* pop_ball           - Lasserre relaxation on the unit ball with a weighted SOS
                       multiplier: p - gamma = s0 + s1 (1 - |x|^2) (Section II-B,
                       constrained POP; Section VI, weighted SOS).
* example_pop        - the quartic test POP of Section VII-A on the unit ball.
* lyapunov           - global Lyapunov search for a cubic vector field
                       (Section II-B, the Lyapunov SOS program) with a quartic V.
* lyapunov_local     - local stability on a ball with a quadratic V and a quadratic
                       multiplier (Section VII-B, Table II's programs).
* small closed forms - univariate, bivariate, separable, infeasible and unbounded
                       programs whose answers are known without any solver.
"""
from __future__ import annotations

from math import comb
from typing import List, Optional, Sequence

import numpy as np

from .poly import Poly, monomials
from .sdp import ConicProblem, SOSEquation, build_sos_sdp


# ---------------------------------------------------------------- helpers
def _sum_sq(n: int, scale: float = 1.0) -> Poly:
    p = Poly(n)
    for i in range(n):
        p = p + Poly.var(n, i, 2).scale(scale)
    return p


def pop_from_poly(p: Poly, half_degree: int, meta: Optional[dict] = None) -> ConicProblem:
    """max gamma s.t. p - gamma in Sigma[x]_{n,2d}; cost -gamma on the single free variable."""
    n = p.n
    eq = SOSEquation(row_degree=2 * half_degree, g0=p, g={0: Poly.const(n, 1.0)},
                     blocks=[(half_degree, Poly.const(n, 1.0))])
    md = {"kind": "pop", "gamma_index": 0, "n_vars": n, "half_degree": half_degree}
    md.update(meta or {})
    return build_sos_sdp(n, 1, [-1.0], [eq], md)


def ball_form_widths(n: int, half_degree: int):
    """Low-rank widths k (columns of A_f: free variables plus non-orthogonal columns, counted
    over lower triangles) of the ball POP's two forms, and the number of rows m of the weighted
    form.  Weighted (Section VI): gamma plus the multiplier's Gram block, 1 + N1 (N1 + 1) / 2
    with N1 = C(n + d - 1, d - 1).  Extra polynomial (Section II-B): gamma plus the coefficients
    of r(x), 1 + C(n + 2d - 2, 2d - 2)."""
    N1 = comb(n + half_degree - 1, half_degree - 1)
    return 1 + N1 * (N1 + 1) // 2, 1 + comb(n + 2 * half_degree - 2, 2 * half_degree - 2), \
        comb(n + 2 * half_degree, 2 * half_degree)


def ball_pop_from_poly(p: Poly, half_degree: int, meta: Optional[dict] = None,
                       form: str = "weighted") -> ConicProblem:
    """max gamma s.t. p - gamma = s0 + s1 (1 - |x|^2); s0 of degree 2d, s1 of degree 2d-2.

    form "weighted": the multiplier s1 enters as a weighted Gram block (Section VI): its columns
    carry several nonzeros and join A_f.  form "extra": the multiplier is an extra polynomial
    r(x) with free coefficients, p - gamma - r (1 - |x|^2) = s0 and r = s1 (Section II-B), so every
    Gram column has one nonzero and A_f is gamma plus r's coefficients.  form "auto": the form
    with the smaller A_f width (the matrix inversion lemma's small system; Section VI's advantage
    condition compares that width with m), the weighted one on a tie (it has fewer rows)."""
    n = p.n
    ball = Poly.const(n, 1.0) - _sum_sq(n)
    kw, ke, m = ball_form_widths(n, half_degree)
    if form == "auto":
        form = "weighted" if kw <= ke else "extra"
    md = {"kind": "ball_pop", "gamma_index": 0, "n_vars": n, "half_degree": half_degree, "form": form,
          "k_weighted": kw, "k_extra": ke, "m_weighted": m}
    md.update(meta or {})
    if form == "weighted":
        eq = SOSEquation(row_degree=2 * half_degree, g0=p, g={0: Poly.const(n, 1.0)},
                         blocks=[(half_degree, Poly.const(n, 1.0)), (half_degree - 1, ball)])
        return build_sos_sdp(n, 1, [-1.0], [eq], md)
    if form != "extra":
        raise ValueError(f"unknown form {form!r}")
    rmons = monomials(n, 2 * half_degree - 2)
    t = 1 + len(rmons)
    g1 = {0: Poly.const(n, 1.0)}
    g2 = {}
    for k, e in enumerate(rmons):
        mk = Poly(n, {tuple(e): 1.0})
        g1[1 + k] = mk * ball          # p - gamma - sum_k r_k m_k (1 - |x|^2) = s0
        g2[1 + k] = mk.scale(-1.0)     # 0 - sum_k r_k (-m_k) = r = s1
    eq1 = SOSEquation(row_degree=2 * half_degree, g0=p, g=g1, blocks=[(half_degree, Poly.const(n, 1.0))])
    eq2 = SOSEquation(row_degree=2 * half_degree - 2, g0=Poly(n), g=g2, blocks=[(half_degree - 1, Poly.const(n, 1.0))])
    return build_sos_sdp(n, t, [-1.0] + [0.0] * (t - 1), [eq1, eq2], md)


# ---------------------------------------------------------------- quartic POPs
def quartic_poly(n: int, rng: np.random.Generator, cross_std: float = 0.0) -> Poly:
    """sum_i x_i^4 + N(0,1) on every monomial of degree <= 3 (+ N(0,cross_std) on quartic cross terms)."""
    terms = {}
    low = monomials(n, 3)
    coef = rng.standard_normal(len(low))
    for e, c in zip(low, coef):
        terms[e] = c
    if cross_std > 0.0:
        quart = [e for e in monomials(n, 4, min_degree=4) if max(e) < 4]
        cc = rng.standard_normal(len(quart)) * cross_std
        for e, c in zip(quart, cc):
            terms[e] = c
    for i in range(n):
        e = [0] * n
        e[i] = 4
        terms[tuple(e)] = 1.0
    return Poly(n, terms)


def pop_unconstrained(n: int, seed: int, cross_std: float = 0.0) -> ConicProblem:
    """Unconstrained quartic POP relaxation (one Gram block of size C(n+2,2))."""
    rng = np.random.default_rng(seed)
    p = quartic_poly(n, rng, cross_std)
    return pop_from_poly(p, 2, {"family": "pop_unconstrained", "seed": seed, "cross_std": cross_std})


def variable_scale(p: Poly, starts: int = 4, seed: int = 12345) -> float:
    """Scale s for the substitution x = s y: the largest |x_i| of the best local minimiser of p
    found by BFGS from a few seeded starts (at least 1).  A modelling step, like the variable
    scaling of POP modelling tools; it leaves the relaxation's optimum unchanged (gamma = s^4
    gamma_y for a quartic written as p(s y) / s^4)."""
    from scipy.optimize import minimize
    n = p.n
    E = np.array([e for e, _ in p.items()], dtype=float)
    C = np.array([c for _, c in p.items()])

    def f(x):
        return float(C @ np.prod(x[None, :] ** E, axis=1))

    def g(x):
        out = np.zeros(n)
        for i in range(n):
            Ei = E.copy()
            mask = Ei[:, i] > 0
            coef = C[mask] * Ei[mask, i]
            Ei = Ei[mask]
            Ei[:, i] -= 1
            out[i] = coef @ np.prod(x[None, :] ** Ei, axis=1)
        return out

    rng = np.random.default_rng(seed)
    best, xb = np.inf, np.ones(n)
    for _ in range(starts):
        r = minimize(f, rng.standard_normal(n), jac=g, method="BFGS", options={"maxiter": 500})
        if r.fun < best:
            best, xb = r.fun, r.x
    return max(1.0, float(np.abs(xb).max()))


def scaled_quartic(p: Poly, s: float) -> Poly:
    """p(s y) / s^4 as a polynomial in y."""
    return Poly(p.n, {e: c * s ** (sum(e) - 4) for e, c in p.items()})


def pop_batch_member(seed: int, scaled: bool = True) -> ConicProblem:
    """Batch member: n ~ U{6..16} drawn first from the seed's stream, then the quartic POP at that n.

    With scaled=True the POP is written in y = x / s (see variable_scale); the solver then
    returns gamma_y and gamma = s^4 gamma_y (meta["gamma_scale"])."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(6, 17))
    p = quartic_poly(n, rng, 0.0)
    s = variable_scale(p) if scaled else 1.0
    q = scaled_quartic(p, s) if scaled else p
    return pop_from_poly(q, 2, {"family": "pop_batch", "seed": seed, "n_vars": n, "scale": s,
                                "gamma_scale": s ** 4})


def pop_ball(n: int, seed: int, form: str = "weighted", half_degree: int = 2) -> ConicProblem:
    """POP on the unit ball, N(0,1) on every monomial of degree <= 4 (quartic p), relaxation of
    order 2d = 2 half_degree; the multiplier in the given form (see ball_pop_from_poly)."""
    rng = np.random.default_rng(seed)
    mons = monomials(n, 4)
    coef = rng.standard_normal(len(mons))
    p = Poly(n, dict(zip(mons, coef)))
    return ball_pop_from_poly(p, half_degree, {"family": "pop_ball", "seed": seed}, form=form)


def example_pop_poly(n: int) -> Poly:
    """sum_{i<j} (x_i x_j + x_i^2 x_j - x_j^3 - x_i^2 x_j^2)  (Section VII-A test polynomial)."""
    p = Poly(n)
    for j in range(n):
        for i in range(j):
            xi, xj = Poly.var(n, i), Poly.var(n, j)
            p = p + xi * xj + Poly.var(n, i, 2) * xj - Poly.var(n, j, 3) - Poly.var(n, i, 2) * Poly.var(n, j, 2)
    return p


def example_pop(n: int) -> ConicProblem:
    """Order-2 (2d = 4) Lasserre relaxation of the Section VII-A POP on the unit ball."""
    return ball_pop_from_poly(example_pop_poly(n), 2, {"family": "example_pop"})


# ---------------------------------------------------------------- Lyapunov family
def lyapunov_field(n: int, rng: np.random.Generator):
    """f_i = -x_i - x_i^3 + sigma * sum_alpha c_{i,alpha} x^alpha over all quadratic monomials."""
    sigma = float(rng.uniform(0.0, 0.5))
    quad = monomials(n, 2, min_degree=2)
    coef = rng.standard_normal((n, len(quad)))
    f = []
    for i in range(n):
        fi = -Poly.var(n, i) - Poly.var(n, i, 3)
        for e, c in zip(quad, coef[i]):
            fi = fi + Poly.mono(e, sigma * c)
        f.append(fi)
    return sigma, coef, f


def lyapunov_from_field(n: int, f: Sequence[Poly], eps: float = 1.0, meta: Optional[dict] = None) -> ConicProblem:
    """find V = sum_i u_i x^{a_i} (2 <= |a_i| <= 4) with V - eps|x|^2 SOS and -grad V . f - eps|x|^2 SOS."""
    vmons = monomials(n, 4, min_degree=2)
    t = len(vmons)
    neg_sq = -_sum_sq(n, eps)
    g1 = {i: Poly.mono(e, -1.0) for i, e in enumerate(vmons)}
    g2 = {}
    for i, e in enumerate(vmons):
        mono = Poly.mono(e)
        acc = Poly(n)
        for k in range(n):
            acc = acc + mono.diff(k) * f[k]
        g2[i] = acc
    eq1 = SOSEquation(row_degree=4, g0=neg_sq, g=g1, blocks=[(2, Poly.const(n, 1.0))])
    eq2 = SOSEquation(row_degree=6, g0=neg_sq, g=g2, blocks=[(3, Poly.const(n, 1.0))])
    md = {"kind": "lyapunov", "n_vars": n, "eps": eps, "v_monomials": t}
    md.update(meta or {})
    return build_sos_sdp(n, t, np.zeros(t), [eq1, eq2], md)


def lyapunov(seed: int, n: int = 6, eps: float = 1.0) -> ConicProblem:
    rng = np.random.default_rng(seed)
    sigma, coef, f = lyapunov_field(n, rng)
    features = np.concatenate([[sigma], (sigma * coef).reshape(-1)])
    return lyapunov_from_field(n, f, eps, {"family": "lyapunov", "seed": seed, "sigma": sigma,
                                           "features": features})


def lyapunov_features(seed: int, n: int = 6) -> np.ndarray:
    """The warm-start model's input for one instance: [sigma, sigma * c_{i,alpha}] (1 + n * C(n+1,2))."""
    rng = np.random.default_rng(seed)
    sigma = float(rng.uniform(0.0, 0.5))
    quad = monomials(n, 2, min_degree=2)
    coef = rng.standard_normal((n, len(quad)))
    return np.concatenate([[sigma], (sigma * coef).reshape(-1)])


# ---------------------------------------------------------------- local Lyapunov family (Table II)
def local_field(n: int, rng: np.random.Generator, terms: int = 2, scale: float = 1.0):
    """A cubic vector field with a linearly stable equilibrium at the origin (Section VII-B):
    f(x) = J x + (per component) `terms` random quadratic and `terms` random cubic monomials with
    N(0, scale^2) coefficients, J = -I + N(0, 1/(4n)) entries, redrawn until every eigenvalue of J
    has real part below -0.1.  Returns (J, f)."""
    while True:
        J = -np.eye(n) + rng.standard_normal((n, n)) * (0.5 / np.sqrt(n))
        if np.max(np.linalg.eigvals(J).real) < -0.1:
            break
    quad = monomials(n, 2, min_degree=2)
    cub = monomials(n, 3, min_degree=3)
    f = []
    for i in range(n):
        fi = Poly(n)
        for j in range(n):
            fi = fi + Poly.var(n, j).scale(J[i, j])
        for pool in (quad, cub):
            for k in rng.choice(len(pool), size=min(terms, len(pool)), replace=False):
                fi = fi + Poly.mono(pool[k], scale * float(rng.standard_normal()))
        f.append(fi)
    return J, f


def local_lyapunov_from_field(n: int, f: Sequence[Poly], radius2: float = 0.1, eps: float = 1.0,
                              meta: Optional[dict] = None) -> ConicProblem:
    """Local stability on the ball D = {x : radius2 - |x|^2 >= 0} with a quadratic Lyapunov function
    (Section II-B's Lyapunov conditions, Section VII-B's experiment): find V = x^T Q x and a
    quadratic multiplier s with

        V - eps |x|^2                        SOS   (Gram basis x_1..x_n),
        s                                    SOS   (Gram basis x_1..x_n),
        -grad V . f - eps |x|^2 - s (radius2 - |x|^2)   SOS   (Gram basis: monomials of degree 1..2),

    so that V > 0 and dV/dt < 0 on D away from the origin.  The coefficients of V and of s are the
    free variables (the multiplier enters as an extra polynomial, Section II-B), t = n (n + 1); rows
    match the coefficients that can occur: degree 2 for the first two identities, degrees 2..4 for
    the third.  Sizes: N = C(n+2, 2) - 1, m = C(n+4, 4) + n^2 - 1, as in Table II.  Feasibility
    problem (c = 0)."""
    quad = monomials(n, 2, min_degree=2)
    nq = len(quad)
    t = 2 * nq
    neg_sq = -_sum_sq(n, eps)
    ball = Poly.const(n, radius2) - _sum_sq(n)
    g1 = {i: Poly.mono(e, -1.0) for i, e in enumerate(quad)}
    g2 = {nq + i: Poly.mono(e, -1.0) for i, e in enumerate(quad)}
    g3 = {}
    for i, e in enumerate(quad):
        mono = Poly.mono(e)
        acc = Poly(n)
        for k in range(n):
            acc = acc + mono.diff(k) * f[k]
        g3[i] = acc                                  # -u_i * (grad x^e . f) on the left side
        g3[nq + i] = mono * ball                     # -w_i * x^e (radius2 - |x|^2)
    one = Poly.const(n, 1.0)
    eq1 = SOSEquation(row_degree=2, row_min_degree=2, g0=neg_sq, g=g1, blocks=[(1, one, 1)])
    eq2 = SOSEquation(row_degree=2, row_min_degree=2, g0=Poly(n), g=g2, blocks=[(1, one, 1)])
    eq3 = SOSEquation(row_degree=4, row_min_degree=2, g0=neg_sq, g=g3, blocks=[(2, one, 1)])
    md = {"kind": "lyapunov_local", "n_vars": n, "eps": eps, "radius2": radius2, "v_monomials": nq}
    md.update(meta or {})
    return build_sos_sdp(n, t, np.zeros(t), [eq1, eq2, eq3], md)


def lyapunov_local(n: int, seed: int, terms: int = 2, scale: float = 1.0) -> ConicProblem:
    """Table II's program for a random cubic system with n states (local_field)."""
    rng = np.random.default_rng(seed)
    J, f = local_field(n, rng, terms, scale)
    return local_lyapunov_from_field(n, f, meta={"family": "lyapunov_local", "seed": seed, "J": J, "f": f})


# ---------------------------------------------------------------- closed-form cases
def univariate(coeffs_low_to_high: Sequence[float]) -> ConicProblem:
    """max gamma s.t. p - gamma SOS for p(x) = sum_k a_k x^k of even degree."""
    deg = len(coeffs_low_to_high) - 1
    if deg % 2:
        raise ValueError("even degree required")
    p = Poly(1, {(k,): float(a) for k, a in enumerate(coeffs_low_to_high)})
    return pop_from_poly(p, deg // 2, {"family": "univariate"})


def univariate_stack(polys: Sequence[Sequence[float]]) -> ConicProblem:
    """max sum_i gamma_i s.t. p_i - gamma_i SOS for several univariate polynomials at once: one
    SOS equation, free variable and Gram block per polynomial (a program with as many PSD blocks
    as polynomials); the optimum is gamma_i = min p_i for each."""
    eqs = []
    for i, a in enumerate(polys):
        deg = len(a) - 1
        if deg % 2:
            raise ValueError("even degrees only")
        p = Poly(1, {(k,): float(c) for k, c in enumerate(a) if c != 0.0})
        eqs.append(SOSEquation(row_degree=deg, g0=p, g={i: Poly.const(1, 1.0)}, blocks=[(deg // 2, Poly.const(1, 1.0))]))
    return build_sos_sdp(1, len(polys), [-1.0] * len(polys), eqs, {"kind": "univariate_stack", "count": len(polys)})


def bivariate_quartic(seed: int) -> ConicProblem:
    """x^4 + y^4 + N(0,1) on every monomial of degree <= 3 in two variables."""
    rng = np.random.default_rng(seed)
    return pop_from_poly(quartic_poly(2, rng, 0.0), 2, {"family": "bivariate", "seed": seed})


def separable_quartic(n: int, seed: int):
    """p = sum_i q_i(x_i) with q_i = x^4 + a3 x^3 + a2 x^2 + a1 x; returns (problem, list of q_i coeffs)."""
    rng = np.random.default_rng(seed)
    qs = []
    terms = {}
    for i in range(n):
        a = rng.standard_normal(3)
        qs.append(np.array([0.0, a[0], a[1], a[2], 1.0]))
        for k, ak in zip((1, 2, 3, 4), (a[0], a[1], a[2], 1.0)):
            e = [0] * n
            e[i] = k
            terms[tuple(e)] = ak
    return pop_from_poly(Poly(n, terms), 2, {"family": "separable", "seed": seed}), qs


def infeasible_pop() -> ConicProblem:
    """max gamma s.t. -x^2 - gamma SOS: no Gram matrix can match a negative x^2 coefficient."""
    return pop_from_poly(Poly(1, {(2,): -1.0}), 1, {"family": "infeasible"})


def unbounded_pop() -> ConicProblem:
    """min gamma s.t. x^2 - gamma SOS (cost +gamma): gamma can go to -infinity."""
    p = Poly(1, {(2,): 1.0})
    eq = SOSEquation(row_degree=2, g0=p, g={0: Poly.const(1, 1.0)}, blocks=[(1, Poly.const(1, 1.0))])
    return build_sos_sdp(1, 1, [1.0], [eq], {"family": "unbounded", "gamma_index": 0})


def shape_counts(n: int, two_d: int):
    """(N, m) = (C(n+d, d), C(n+2d, 2d)) for the full monomial basis (Section II-C)."""
    d = two_d // 2
    return comb(n + d, d), comb(n + two_d, two_d)


FAMILIES = {
    "c1": lambda seed=0: pop_unconstrained(4, seed),
    "c2": lambda seed=0: pop_unconstrained(20, seed, cross_std=0.1),
    "c3": lambda seed=0: pop_ball(16, seed),
    "c4": pop_batch_member,
    "c5": lyapunov,
}
