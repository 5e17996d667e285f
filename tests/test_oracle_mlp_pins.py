"""Pins of the FP64 oracle network (warm-start MLP): closed-form networks and finite
differences of its own forward pass for the gradient."""
import numpy as np

import oracle as O


def _pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def test_absolute_value_network():
    """|x| = relu(x) + relu(-x): widths (1, 2, 1) with W1 = [1, -1], W2 = [1, 1]."""
    params = _pack([(np.array([[1.0], [-1.0]]), np.zeros(2)), (np.array([[1.0, 1.0]]), np.zeros(1))])
    x = np.linspace(-3, 3, 13)[:, None]
    np.testing.assert_allclose(O.mlp_forward([1, 2, 1], params, x)[:, 0], np.abs(x[:, 0]), rtol=0, atol=1e-15)


def test_linear_output_layer_and_bias():
    """One layer is affine: y = W x + b (no ReLU on the output layer)."""
    rng = np.random.default_rng(0)
    W, b = rng.standard_normal((3, 4)), rng.standard_normal(3)
    x = rng.standard_normal((5, 4))
    np.testing.assert_allclose(O.mlp_forward([4, 3], _pack([(W, b)]), x), x @ W.T + b, rtol=1e-14)


def test_hidden_relu_clips_negative_preactivations():
    """A hidden unit with a negative pre-activation contributes nothing."""
    params = _pack([(np.array([[1.0], [1.0]]), np.array([0.0, -10.0])), (np.array([[2.0, 5.0]]), np.array([0.5]))])
    x = np.array([[1.0], [3.0]])
    np.testing.assert_allclose(O.mlp_forward([1, 2, 1], params, x)[:, 0], 2.0 * x[:, 0] + 0.5)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    widths = [5, 7, 6, 3]
    n = O.mlp_param_count(widths)
    p = rng.standard_normal(n) * 0.5
    x = rng.standard_normal((9, 5))
    t = rng.standard_normal((9, 3))
    wt = rng.uniform(0.5, 2.0, (9, 3))
    loss, g = O.mlp_backward(widths, p, x, t, wt)
    y = O.mlp_forward(widths, p, x)
    assert loss == np.sum(0.5 * wt * (y - t) ** 2)
    h = 1e-6
    for i in rng.choice(n, 40, replace=False):
        e = np.zeros(n)
        e[i] = h
        lp, _ = O.mlp_backward(widths, p + e, x, t, wt)
        lm, _ = O.mlp_backward(widths, p - e, x, t, wt)
        assert abs((lp - lm) / (2 * h) - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
