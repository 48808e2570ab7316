"""GPU solution post-processing (sos_psd_factor and paper_1708_04174_amd.postprocess) against
LAPACK on the same Gram matrix and against the oracle's own post-processing."""
import numpy as np
import pytest

from oracle import postprocess as OP
from oracle.admm import SOLVED, Oracle
from sosgen import Poly, families as F
from sosgen.poly import monomials

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_04174_amd import binding
    binding.load()
    return binding


def _solve(B, prob, tol, max_iters):
    w = B.setup_problem(prob, B.sos_default_settings(tol=tol, max_iters=max_iters))
    inf = B.sos_solve(w)
    return w, inf


@pytest.mark.parametrize("dual", [False, True])
def test_factor_matches_lapack_on_the_same_matrix(B, dual):
    prob = F.FAMILIES["c1"](0)
    w, inf = _solve(B, prob, 1e-6, 5000)
    assert inf["status"] == 1
    x, y, z = B.sos_get_solution(w)
    N = prob.psd_dims[0]
    W = (z if dual else x)[1:].reshape(N, N, order="F")
    lam, V = B.sos_psd_factor(w, 0, dual=dual)
    w.free()
    ref = np.linalg.eigvalsh(W)
    scale = max(1.0, np.abs(ref).max())
    print(f"[post] dual={dual}: max |lambda - lapack| {np.abs(np.sort(lam) - ref).max():.2e} (scale {scale:.2e})")
    assert np.abs(np.sort(lam) - ref).max() <= 1e-10 * scale
    assert np.abs(V.T @ V - np.eye(N)).max() <= 1e-10
    assert np.abs((V * lam) @ V.T - W).max() <= 1e-10 * scale


@pytest.mark.parametrize("seed", [0, 1])
def test_sos_decomposition_against_the_oracle(B, seed):
    from paper_1708_04174_amd import postprocess as PP
    prob = F.FAMILIES["c1"](seed)
    n = prob.meta["n_vars"]
    w, inf = _solve(B, prob, 1e-8, 40000)
    assert inf["status"] == 1
    dec = PP.sos_decomposition(w, prob.b, monomials(n, 4), monomials(n, 2))
    w.free()
    r = Oracle.from_problem(prob).solve(tol=1e-8, max_iters=40000)
    assert r.status == SOLVED
    lam, V = OP.gram_factors(r.x[1:].reshape(prob.psd_dims[0], -1, order="F"))
    p = {e: float(v) for e, v in zip(monomials(n, 4), prob.b) if v != 0.0}
    res_o = OP.identity_residual(p, r.x[0], OP.square_sum(OP.sos_terms(lam, V, monomials(n, 2))), n)
    bound = 1e-8 * (1 + np.linalg.norm(prob.b)) * 10
    print(f"[post] c1 seed {seed}: gamma gpu {dec.gamma:.9f} oracle {r.x[0]:.9f}; identity residual gpu "
          f"{dec.residual:.2e} oracle {res_o:.2e} (bound {bound:.1e}); squares {len(dec.weights)}")
    assert dec.residual <= bound and res_o <= bound
    assert abs(dec.gamma - r.x[0]) <= 1e-6 * max(1.0, abs(r.x[0]))


def _bivariate():
    n = 2
    s = Poly.var(n, 0) - Poly.const(n, 0.5)
    t = Poly.var(n, 1) + Poly.const(n, 0.3)
    return F.pop_from_poly(s * s + t * t + s * s * s * s + (s * s) * (t * t) + t * t * t * t, 2), np.array([0.5, -0.3])


def test_minimiser_from_the_dual_against_the_oracle(B):
    from paper_1708_04174_amd import postprocess as PP
    prob, xstar = _bivariate()
    w, inf = _solve(B, prob, 1e-9, 80000)
    assert inf["status"] == 1
    x, ratio = PP.minimiser(w, monomials(2, 4), 2)
    w.free()
    r = Oracle.from_problem(prob).solve(tol=1e-9, max_iters=80000)
    xo, ro = OP.extract_minimiser(OP.moments(r.y, monomials(2, 4)), monomials(2, 2), 2)
    print(f"[post] bivariate: gpu x* {x} ratio {ratio:.1e}; oracle x* {xo} ratio {ro:.1e}")
    assert ratio < 1e-3 and np.allclose(x, xstar, atol=1e-3) and np.allclose(x, xo, atol=1e-3)


def test_two_minimisers_are_flagged(B):
    from paper_1708_04174_amd import postprocess as PP
    w, inf = _solve(B, F.univariate([1.0, 0.0, -2.0, 0.0, 1.0]), 1e-9, 40000)
    _, ratio = PP.minimiser(w, monomials(1, 4), 1)
    w.free()
    assert ratio > 0.1


def test_factor_argument_errors(B):
    w, _ = _solve(B, F.FAMILIES["c1"](0), 1e-4, 2000)
    with pytest.raises(B.SosError) as e:
        B.sos_psd_factor(w, 1)
    assert e.value.code == B.SOS_E_INVAL
    w.free()
