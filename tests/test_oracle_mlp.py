"""Pins of the FP64 cost-model MLP reference."""
import numpy as np

from oracle import mlp


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    F, B = 12, 16
    p = mlp.init(F, 16, 16, seed=1)
    for k in ("b1", "b2"):
        p[k] = rng.normal(0, 0.1, size=p[k].shape)
    X = rng.normal(size=(B, F))
    t = rng.normal(size=B)
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, y, t)
    h = 1e-6
    for name in mlp.NAMES:
        W = p[name]
        for idx in list(np.ndindex(W.shape))[:: max(1, W.size // 25)]:
            old = W[idx]
            W[idx] = old + h
            lp = mlp.loss(p, X, t)
            W[idx] = old - h
            lm = mlp.loss(p, X, t)
            W[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd))


def test_last_layer_gradient_vanishes_at_least_squares():
    """For fixed hidden features the loss is quadratic in (W3, b3); its
    gradient must vanish at the ordinary least-squares solution of
    y ~ h2 w + b (numpy lstsq) and equal (2/B) A^T (A w - t) elsewhere."""
    rng = np.random.default_rng(2)
    F, B = 4, 64
    p = mlp.init(F, 8, 8, seed=3)
    X = rng.normal(size=(B, F))
    t = rng.normal(size=B)
    _, cache = mlp.forward(p, X)
    A = np.hstack([cache[4], np.ones((B, 1))])
    sol, *_ = np.linalg.lstsq(A, t, rcond=None)
    p["W3"][0], p["b3"][0] = sol[:-1], sol[-1]
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, y, t)
    assert np.max(np.abs(g["W3"])) < 1e-10 and abs(g["b3"][0]) < 1e-10
    w = rng.normal(size=A.shape[1])
    p["W3"][0], p["b3"][0] = w[:-1], w[-1]
    y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, y, t)
    ref = 2.0 / B * A.T @ (A @ w - t)
    assert np.allclose(np.concatenate([g["W3"][0], g["b3"]]), ref, atol=1e-12)


def test_adam_first_step_is_signed_lr():
    """Adam's bias correction makes the first update exactly -lr*sign(g)
    (up to eps) for every weight."""
    rng = np.random.default_rng(4)
    p = mlp.init(6, 8, 8, seed=5)
    before = {k: v.copy() for k, v in p.items()}
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    mlp.adam_step(p, g, {}, lr=1e-2, eps=1e-12)
    for k in mlp.NAMES:
        assert np.allclose(p[k] - before[k], -1e-2 * np.sign(g[k]), atol=1e-9)
