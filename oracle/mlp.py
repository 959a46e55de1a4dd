"""Plain FP64 definitions for the distant-pair surrogate (features, MLP, Adam).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper contains no learned component; the surrogate is a project
addition that predicts the pair energy of Eq. ED2 for distant pairs.  Its
definition here is the specification the GPU kernels are checked against.

Readings (the paper is silent on all of them):

* Per-fragment invariants of the Coulomb moments d^x = B^x : D^x (the same
  moments that drive the field of Eqs. wc / dp2e):
  u^x = [d.G^k.d for k = 0..3] + [(q_k . d)^2 for the 4 eigenvectors q_k of G
  with the largest eigenvalues]  (8 numbers, unchanged by eigenvector signs).
* Pair features (17): [R_xy (bohr), u^x_k + u^y_k (8), u^x_k * u^y_k (8)],
  symmetric under x <-> y; each feature is standardised with a mean and
  standard deviation fixed from the training set.
* Target: E2_xy * R_xy^2 (bohr^2), standardised; since every integral of the
  pair scales as 1/R_xy at fixed orbitals, E2 R^2 removes the leading
  distance dependence.
* Network: 17 -> 128 -> 128 -> 1, SiLU after the first two layers.
  Weights W_l are stored [out][in].  Loss: mean squared error.
* Optimiser: Adam with bias correction.
"""
from __future__ import annotations

import numpy as np

LAYERS = (17, 128, 128, 1)


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def fragment_invariants(d: np.ndarray, G: np.ndarray) -> np.ndarray:
    """u^x from the moment vector d (length P0) and the class-0 coupling G."""
    u = np.empty(8)
    v = d.copy()
    for k in range(4):
        u[k] = d @ v           # d . G^k . d
        v = G @ v
    w, q = np.linalg.eigh(G)
    top = q[:, ::-1][:, :4]    # eigenvectors of the 4 largest eigenvalues
    u[4:] = (top.T @ d) ** 2
    return u


def pair_features(r_bohr: float, ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
    return np.concatenate([[r_bohr], ux + uy, ux * uy])


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


def init_params(rng: np.random.Generator):
    """Kaiming-uniform style init (bounds 1/sqrt(fan_in)); biases zero."""
    p = {}
    for l in range(3):
        fi, fo = LAYERS[l], LAYERS[l + 1]
        bound = 1.0 / np.sqrt(fi)
        p[f"W{l}"] = rng.uniform(-bound, bound, size=(fo, fi))
        p[f"b{l}"] = np.zeros(fo)
    return p


def forward(p, X):
    """Returns (y [N], cache) for inputs X [N, 17]."""
    z0 = X @ p["W0"].T + p["b0"]
    h0 = silu(z0)
    z1 = h0 @ p["W1"].T + p["b1"]
    h1 = silu(z1)
    y = (h1 @ p["W2"].T + p["b2"])[:, 0]
    return y, (X, z0, h0, z1, h1)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - t) ** 2))


def backward(p, X, t):
    """Gradients of the mean squared error with respect to every parameter."""
    y, (X, z0, h0, z1, h1) = forward(p, X)
    n = X.shape[0]
    gy = (2.0 / n) * (y - t)                   # dL/dy
    g = {}
    g["W2"] = gy[None, :] @ h1                 # [1,128]
    g["b2"] = np.array([gy.sum()])
    gh1 = gy[:, None] @ p["W2"]                # [N,128]
    gz1 = gh1 * silu_grad(z1)
    g["W1"] = gz1.T @ h0
    g["b1"] = gz1.sum(axis=0)
    gh0 = gz1 @ p["W1"]
    gz0 = gh0 * silu_grad(z0)
    g["W0"] = gz0.T @ X
    g["b0"] = gz0.sum(axis=0)
    return g


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step index t >= 1) of every parameter, in place."""
    for k in p:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** t)
        vh = v[k] / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
