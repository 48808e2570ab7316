"""Seeded synthetic SOS programs, written out as conic data (A, b, c, K).

This package turns polynomial problems into the standard-form SDP of the
paper (Section III): min c^T xi  s.t.  A xi = b,  xi in K = R^t x S^{N_1}_+ x ...,
with every PSD block stored as the column-stacked vec of the Gram matrix.
It holds no part of the ADMM method: both the CPU oracle and the GPU library
take its output as plain input data.
"""
from .poly import monomials, n_monomials, Poly
from .sdp import ConicProblem, SOSEquation, build_sos_sdp
from . import families

__all__ = ["monomials", "n_monomials", "Poly", "ConicProblem", "SOSEquation",
           "build_sos_sdp", "families"]
