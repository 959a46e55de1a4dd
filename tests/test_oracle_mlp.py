"""Pins for the surrogate's CPU oracle (features, network, gradients, Adam)."""
import numpy as np
import pytest

from oracle import mlp


def _params(seed=0):
    return mlp.init_params(np.random.default_rng(seed))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = _params(1)
    for k in p:  # non-zero biases so that their gradients are exercised
        if k.startswith("b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((7, 17))
    t = rng.standard_normal(7)
    g = mlp.backward(p, X, t)
    h = 1e-6
    for k in p:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h; lp = mlp.loss(p, X, t)
            flat[i] = old - h; lm = mlp.loss(p, X, t)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            assert abs(num - g[k].ravel()[i]) <= 1e-7 + 1e-6 * abs(num), (k, i)


def test_silu_derivative():
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    num = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.silu_grad(z), num, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(mlp.silu(np.array([0.0])), [0.0])


def test_adam_first_step_is_signed_lr():
    """At t = 1 the bias-corrected moments are g and g^2, so the update is
    -lr g / (|g| + eps)."""
    p = {"w": np.array([0.5, -1.0, 2.0])}
    g = {"w": np.array([3.0, -0.25, 1e-3])}
    m = {"w": np.zeros(3)}; v = {"w": np.zeros(3)}
    mlp.adam_step(p, g, m, v, 1, lr=0.01, eps=1e-8)
    exp = np.array([0.5, -1.0, 2.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    np.testing.assert_allclose(p["w"], exp, rtol=1e-14)


def test_invariants():
    rng = np.random.default_rng(2)
    q, _ = np.linalg.qr(rng.standard_normal((72, 72)))
    lam = rng.uniform(0.1, 1, 72)
    G = (q * lam) @ q.T; G = 0.5 * (G + G.T)
    d = rng.standard_normal(72)
    u = mlp.fragment_invariants(d, G)
    assert u[0] == pytest.approx(d @ d, rel=1e-14)
    assert u[1] == pytest.approx(d @ G @ d, rel=1e-13)
    assert u[3] == pytest.approx(d @ G @ G @ G @ d, rel=1e-12)
    # projections on the eigenvectors of the largest eigenvalues: they sum to
    # |d|^2 over a full eigenbasis (Parseval); the top four are the largest
    # eigenvalues' (lambda-weighted sum bounded by d.G.d)
    order = np.argsort(lam)[::-1]
    proj = (q[:, order[:4]].T @ d) ** 2
    np.testing.assert_allclose(np.sort(u[4:]), np.sort(proj), rtol=1e-10)
    # sign-invariance: the invariants do not change under d -> -d
    np.testing.assert_allclose(mlp.fragment_invariants(-d, G), u, rtol=1e-14)


def test_pair_features_symmetric():
    rng = np.random.default_rng(3)
    ux, uy = rng.standard_normal(8), rng.standard_normal(8)
    np.testing.assert_array_equal(mlp.pair_features(7.0, ux, uy),
                                  mlp.pair_features(7.0, uy, ux))
    assert mlp.pair_features(7.0, ux, uy).shape == (17,)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((256, 17))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    p = _params(4)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    l0 = mlp.loss(p, X, t)
    for step in range(1, 201):
        g = mlp.backward(p, X, t)
        mlp.adam_step(p, g, m, v, step, lr=3e-3)
    assert mlp.loss(p, X, t) < 0.2 * l0
