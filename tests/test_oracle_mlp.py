"""Pins for the FP64 reference MLP: closed-form GELU values, central finite differences
of the loss, and the closed form of Adam's first step."""
import math

import numpy as np

from oracle import mlp


def test_gelu_closed_forms():
    # gelu(z) = z Phi(z); Phi(1) = 0.841344746068543, Phi(-1) = 1 - Phi(1)
    phi1 = 0.5 * (1 + math.erf(1 / math.sqrt(2)))
    z = np.array([0.0, 1.0, -1.0, 8.0, -8.0])
    g = mlp.gelu(z)
    assert g[0] == 0.0
    assert abs(g[1] - phi1) < 1e-15 and abs(g[2] + (1 - phi1)) < 1e-15
    assert abs(g[3] - 8.0) < 1e-12 and abs(g[4]) < 1e-12
    # derivative against central differences
    zz = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(zz + h) - mlp.gelu(zz - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(zz))) < 1e-8


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    dims = (5, 7, 4)
    n = mlp.num_params(*dims)
    theta = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((6, dims[0]))
    T = rng.standard_normal((6, dims[2]))
    g, L = mlp.gradient(theta, X, T, dims)
    assert abs(L - mlp.loss(theta, X, T, dims)) < 1e-15
    h = 1e-6
    fd = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd[i] = (mlp.loss(theta + e, X, T, dims) - mlp.loss(theta - e, X, T, dims)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-7 * max(1.0, np.max(np.abs(g)))


def test_layout_orders_parameters_as_documented():
    dims = (3, 4, 2)
    theta = np.arange(mlp.num_params(*dims), dtype=float)
    p = mlp.unpack(theta, *dims)
    assert p["W1"].shape == (3, 4) and p["W1"][0, 1] == 1.0 and p["W1"][1, 0] == 4.0
    assert p["b1"][0] == 12.0 and p["W2"][0, 0] == 16.0 and p["b3"][-1] == theta[-1]


def test_adam_first_step_closed_form():
    # bias correction makes the first step lr * g / (|g| + eps)
    g = np.array([2.0, -0.5, 1e-3, 0.0])
    opt = mlp.Adam(4, lr=0.1)
    th = opt.step(np.zeros(4), g)
    assert np.allclose(th, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_training_reduces_loss_on_a_smooth_map():
    rng = np.random.default_rng(1)
    dims = (3, 16, 2)
    X = rng.standard_normal((64, 3))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1], X[:, 2] ** 2], axis=1)
    theta = rng.standard_normal(mlp.num_params(*dims)) * 0.3
    opt = mlp.Adam(theta.size, lr=0.01)
    L0 = mlp.loss(theta, X, T, dims)
    for _ in range(300):
        g, _ = mlp.gradient(theta, X, T, dims)
        theta = opt.step(theta, g)
    assert mlp.loss(theta, X, T, dims) < 0.2 * L0


class _AdamWithoutPowerInBiasCorrection(mlp.Adam):
    """Planted mistake: bias correction by 1 - beta instead of 1 - beta^t."""

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        return theta - self.lr * (self.m / (1 - self.b1)) / (np.sqrt(self.v / (1 - self.b2)) + self.eps)


def _adam_unrolled(gs, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam's parameter after len(gs) steps from 0, each step written in closed form: the
    moment estimates are the bias-normalised geometric averages
    m_hat_t = sum_s b1^(t-s) g_s / sum_s b1^(t-s)  (and likewise v_hat_t with g_s^2, b2),
    since (1 - b) sum_{s<=t} b^(t-s) = 1 - b^t (Kingma & Ba, the bias-correction argument)."""
    gs = np.asarray(gs, dtype=float)
    theta = 0.0
    for t in range(1, len(gs) + 1):
        w1 = b1 ** np.arange(t - 1, -1, -1)
        w2 = b2 ** np.arange(t - 1, -1, -1)
        mh = w1 @ gs[:t] / w1.sum()
        vh = w2 @ gs[:t] ** 2 / w2.sum()
        theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta


def _run(opt_cls, gs, lr=0.05):
    opt = opt_cls(1, lr=lr)
    th = np.zeros(1)
    out = []
    for g in gs:
        th = opt.step(th, np.array([g]))
        out.append(float(th[0]))
    return out


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient the bias-corrected moments are exactly g and g^2 at every t,
    # so each step moves the parameter by lr * g / (|g| + eps), at t = 1, 2, 3, ...
    g, lr = -1.7, 0.05
    got = _run(mlp.Adam, [g] * 5, lr)
    want = [-(t + 1) * lr * g / (abs(g) + 1e-8) for t in range(5)]
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    bad = _run(_AdamWithoutPowerInBiasCorrection, [g] * 5, lr)
    assert np.allclose(bad[0], want[0], rtol=1e-12)        # the mistake is invisible at t = 1 ...
    assert not np.allclose(bad[1:], want[1:], rtol=1e-3)   # ... and caught from t = 2 on


def test_adam_steps_two_and_three_closed_form():
    gs = [2.0, -0.5, 1.25]
    got = _run(mlp.Adam, gs)
    for t in (2, 3):
        assert abs(got[t - 1] - _adam_unrolled(gs[:t], 0.05)) <= 1e-13
    bad = _run(_AdamWithoutPowerInBiasCorrection, gs)
    for t in (2, 3):
        assert abs(bad[t - 1] - _adam_unrolled(gs[:t], 0.05)) > 1e-3
