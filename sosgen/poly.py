"""Monomial bases and sparse polynomials in n variables.

The basis v_d(x) lists all monomials of degree <= d in graded order:
1, x_1, ..., x_n, x_1^2, x_1 x_2, ..., x_n^d  (Section I, the candidate
monomial vector; Section II-A for the multi-index notation N^n_d).
Within one degree the order is lexicographic on the sorted variable
indices, which is what the listing x_1^2, x_1 x_2, ... shows.
"""
from __future__ import annotations

from itertools import combinations_with_replacement
from math import comb
from typing import Dict, Iterable, List, Tuple

Exp = Tuple[int, ...]


def n_monomials(n: int, d: int) -> int:
    """Number of monomials of degree <= d in n variables: C(n+d, d)."""
    return comb(n + d, d)


def monomials(n: int, d: int, min_degree: int = 0) -> List[Exp]:
    """Exponent tuples of all monomials with min_degree <= degree <= d, graded order."""
    out: List[Exp] = []
    for k in range(min_degree, d + 1):
        for idx in combinations_with_replacement(range(n), k):
            e = [0] * n
            for i in idx:
                e[i] += 1
            out.append(tuple(e))
    return out


class Poly:
    """Sparse real polynomial: a dict from exponent tuple to coefficient."""

    __slots__ = ("n", "terms")

    def __init__(self, n: int, terms: Dict[Exp, float] | None = None):
        self.n = n
        self.terms: Dict[Exp, float] = {}
        if terms:
            for e, c in terms.items():
                if len(e) != n:
                    raise ValueError("exponent length mismatch")
                if c != 0.0:
                    self.terms[tuple(e)] = self.terms.get(tuple(e), 0.0) + float(c)

    # -- constructors -------------------------------------------------
    @staticmethod
    def const(n: int, c: float) -> "Poly":
        return Poly(n, {(0,) * n: c})

    @staticmethod
    def var(n: int, i: int, power: int = 1) -> "Poly":
        e = [0] * n
        e[i] = power
        return Poly(n, {tuple(e): 1.0})

    @staticmethod
    def mono(e: Exp, c: float = 1.0) -> "Poly":
        return Poly(len(e), {tuple(e): c})

    # -- arithmetic ---------------------------------------------------
    def copy(self) -> "Poly":
        p = Poly(self.n)
        p.terms = dict(self.terms)
        return p

    def __add__(self, other: "Poly") -> "Poly":
        p = self.copy()
        for e, c in other.terms.items():
            p.terms[e] = p.terms.get(e, 0.0) + c
        p.terms = {e: c for e, c in p.terms.items() if c != 0.0}
        return p

    def __neg__(self) -> "Poly":
        return Poly(self.n, {e: -c for e, c in self.terms.items()})

    def __sub__(self, other: "Poly") -> "Poly":
        return self + (-other)

    def scale(self, s: float) -> "Poly":
        return Poly(self.n, {e: s * c for e, c in self.terms.items()})

    def __mul__(self, other: "Poly") -> "Poly":
        out: Dict[Exp, float] = {}
        for e1, c1 in self.terms.items():
            for e2, c2 in other.terms.items():
                e = tuple(a + b for a, b in zip(e1, e2))
                out[e] = out.get(e, 0.0) + c1 * c2
        return Poly(self.n, out)

    def diff(self, i: int) -> "Poly":
        out: Dict[Exp, float] = {}
        for e, c in self.terms.items():
            if e[i] > 0:
                f = list(e)
                f[i] -= 1
                out[tuple(f)] = out.get(tuple(f), 0.0) + c * e[i]
        return Poly(self.n, out)

    def degree(self) -> int:
        return max((sum(e) for e in self.terms), default=0)

    def coef(self, e: Exp) -> float:
        return self.terms.get(tuple(e), 0.0)

    def __call__(self, x) -> float:
        total = 0.0
        for e, c in self.terms.items():
            t = c
            for xi, k in zip(x, e):
                if k:
                    t *= xi ** k
            total += t
        return total

    def items(self) -> Iterable[Tuple[Exp, float]]:
        return self.terms.items()
