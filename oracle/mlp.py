"""CPU FP64 reference of the warm-start MLP (test infrastructure only).

Only tests/, the smoke check and bench.py's cpu_baseline leg may use oracle/.

The network is the plain definition: input -> H -> H -> output, each hidden layer
Z = X W + b followed by the exact GELU, gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2,
and a linear output layer.  The loss is the mean squared error over all outputs of the
batch; gradients are written out by the chain rule, and Adam follows Kingma & Ba
(bias-corrected first and second moments).  The parameter vector is ordered
[W1, b1, W2, b2, W3, b3] with row-major W (in x out), matching the device library's
documented layout so that gradients can be compared entry by entry.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def _erf(x: np.ndarray) -> np.ndarray:
    from scipy.special import erf
    return erf(x)


def gelu(z: np.ndarray) -> np.ndarray:
    return 0.5 * z * (1.0 + _erf(z / _SQRT2))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


def shapes(n_in: int, n_h: int, n_out: int) -> List[Tuple[str, Tuple[int, ...]]]:
    return [("W1", (n_in, n_h)), ("b1", (n_h,)), ("W2", (n_h, n_h)), ("b2", (n_h,)),
            ("W3", (n_h, n_out)), ("b3", (n_out,))]


def unpack(theta: np.ndarray, n_in: int, n_h: int, n_out: int) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shp in shapes(n_in, n_h, n_out):
        size = int(np.prod(shp))
        out[name] = theta[o:o + size].reshape(shp)
        o += size
    assert o == theta.size
    return out


def pack(parts: Dict[str, np.ndarray], n_in: int, n_h: int, n_out: int) -> np.ndarray:
    return np.concatenate([parts[name].reshape(-1) for name, _ in shapes(n_in, n_h, n_out)])


def num_params(n_in: int, n_h: int, n_out: int) -> int:
    return sum(int(np.prod(s)) for _, s in shapes(n_in, n_h, n_out))


def forward(theta: np.ndarray, X: np.ndarray, dims) -> Tuple[np.ndarray, dict]:
    p = unpack(np.asarray(theta, dtype=np.float64), *dims)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ p["W1"] + p["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = gelu(Z2)
    Y = H2 @ p["W3"] + p["b3"]
    return Y, {"X": X, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2}


def loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray, dims) -> float:
    Y, _ = forward(theta, X, dims)
    return float(np.mean((Y - T) ** 2))


def gradient(theta: np.ndarray, X: np.ndarray, T: np.ndarray, dims) -> Tuple[np.ndarray, float]:
    """d loss / d theta by the chain rule, and the loss."""
    p = unpack(np.asarray(theta, dtype=np.float64), *dims)
    Y, c = forward(theta, X, dims)
    T = np.asarray(T, dtype=np.float64)
    dY = 2.0 * (Y - T) / Y.size
    g = {}
    g["W3"] = c["H2"].T @ dY
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ p["W3"].T) * gelu_grad(c["Z2"])
    g["W2"] = c["H1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"].T) * gelu_grad(c["Z1"])
    g["W1"] = c["X"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return pack(g, *dims), float(np.mean((Y - T) ** 2))


class Adam:
    """theta <- theta - lr * m_hat / (sqrt(v_hat) + eps) with bias-corrected moments."""

    def __init__(self, n: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)
