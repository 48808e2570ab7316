"""Checks a local Lyapunov certificate (Section VII-B's programs, sosgen.families.lyapunov_local)
without the solver: the three polynomial identities evaluated at random points, the Gram blocks'
smallest eigenvalues, the quadratic form's, and dV/dt sampled inside the ball."""
import numpy as np

from sosgen.poly import Poly, monomials


def _basis_values(basis, z):
    return np.array([np.prod(z ** np.array(e)) for e in basis])


def certificate_errors(prob, x, samples=400, seed=1):
    """Returns dict(identity=max relative mismatch of the three identities, gram_min=smallest
    eigenvalue over the Gram blocks relative to their largest, q_min=smallest eigenvalue of Q,
    vdot=max of dV/dt / |x|^2 over points of the ball)."""
    n = prob.meta["n_vars"]
    eps, r2 = prob.meta["eps"], prob.meta["radius2"]
    f = prob.meta["f"]
    quad = monomials(n, 2, min_degree=2)
    nq = len(quad)
    V, s = Poly(n), Poly(n)
    for e, a, b in zip(quad, x[:nq], x[nq:2 * nq]):
        V = V + Poly.mono(e, float(a))
        s = s + Poly.mono(e, float(b))
    Xs = []
    for o, N in zip(prob.block_offsets(), prob.psd_dims):
        X = np.asarray(x[o:o + N * N]).reshape(N, N, order="F")
        Xs.append(0.5 * (X + X.T))
    m1 = monomials(n, 1, min_degree=1)
    m2 = monomials(n, 2, min_degree=1)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(samples):
        z = rng.uniform(-1.0, 1.0, n)
        z2 = float(z @ z)
        vdot = sum(V.diff(k)(z) * f[k](z) for k in range(n))
        b1, b2 = _basis_values(m1, z), _basis_values(m2, z)
        pairs = ((V(z) - eps * z2, b1 @ Xs[0] @ b1), (s(z), b1 @ Xs[1] @ b1),
                 (-vdot - eps * z2 - s(z) * (r2 - z2), b2 @ Xs[2] @ b2))
        for lhs, rhs in pairs:
            worst = max(worst, abs(lhs - rhs) / max(1.0, abs(lhs)))
    gram_min = min(float(np.linalg.eigvalsh(X)[0]) / max(1.0, float(np.max(np.abs(X)))) for X in Xs)
    Q = np.zeros((n, n))
    for e, a in zip(quad, x[:nq]):
        idx = [i for i in range(n) for _ in range(e[i])]
        if idx[0] == idx[1]:
            Q[idx[0], idx[0]] = a
        else:
            Q[idx[0], idx[1]] = Q[idx[1], idx[0]] = a / 2
    vmax = -np.inf
    for _ in range(samples):
        z = rng.standard_normal(n)
        z *= np.sqrt(r2) * rng.uniform() ** (1.0 / n) / np.linalg.norm(z)
        vmax = max(vmax, sum(V.diff(k)(z) * f[k](z) for k in range(n)) / float(z @ z))
    return {"identity": worst, "gram_min": gram_min, "q_min": float(np.linalg.eigvalsh(Q)[0]), "vdot": vmax}
