"""The cost-model oracle pinned to independent facts: central differences,
a network that reduces to a linear model, and Adam's first step."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    D, H, N = 5, 7, 23
    p = mlp.init(D, H, seed=3) + rng.normal(0, 0.1, mlp.nparams(D, H))
    x = rng.normal(0, 1, (N, D))
    t = rng.normal(0, 1, N)
    g, L = mlp.grad(p, x, t, D, H)
    assert abs(L - mlp.loss(p, x, t, D, H)) < 1e-12
    h = 1e-6
    num = np.zeros_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (mlp.loss(p + e, x, t, D, H) - mlp.loss(p - e, x, t, D, H)) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-6 * max(1.0, np.max(np.abs(g)))


def test_all_active_units_reduce_to_a_linear_model():
    """With every pre-activation positive, y = w3.(W2(W1 x + b1) + b2) + b3, so
    the output is exactly affine in x with the product weights."""
    rng = np.random.default_rng(1)
    D, H = 4, 6
    W1 = np.abs(rng.normal(size=(H, D)))
    b1 = np.ones(H)
    W2 = np.abs(rng.normal(size=(H, H)))
    b2 = np.ones(H)
    w3 = rng.normal(size=H)
    b3 = 0.25
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])
    x = np.abs(rng.normal(size=(10, D)))
    y = mlp.forward(p, x, D, H)
    A = w3 @ W2 @ W1
    c = w3 @ (W2 @ b1 + b2) + b3
    assert np.allclose(y, x @ A + c, rtol=1e-12, atol=1e-12)
    # and dL/dW1 = (W2^T w3) outer (sum_s gy_s x_s)
    t = rng.normal(size=10)
    g, _ = mlp.grad(p, x, t, D, H)
    gy = 2 * (y - t) / 10
    gW1 = np.outer(W2.T @ w3, gy @ x)
    assert np.allclose(g[:H * D].reshape(H, D), gW1, rtol=1e-10, atol=1e-12)


def test_adam_first_step_moves_each_weight_by_lr():
    """After bias correction the first Adam step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, 0.01, 0.9, 0.999, 1e-8)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
