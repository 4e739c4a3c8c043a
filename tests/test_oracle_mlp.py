"""Pins of the oracle's perceptron (oracle/mlp.py) against things other than
itself: central differences of the loss, closed forms at special parameter
values, and the closed form of the first Adam step."""
import numpy as np

from oracle import mlp


def tiny(seed=0, n_in=5, n_hid=4, n_out=3, B=3):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.n_params(n_in, n_hid, n_out)) * 0.7
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    return p, X, T, dict(n_in=n_in, n_hid=n_hid, n_out=n_out)


def test_gradient_matches_central_differences():
    p, X, T, kw = tiny()
    g = mlp.loss_grad(p, X, T, **kw)
    h = 1e-6
    num = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        num[k] = (mlp.loss(p + e, X, T, **kw) - mlp.loss(p - e, X, T, **kw)) / (2 * h)
    assert np.max(np.abs(g - num)) < 1e-8


def test_zero_input_weights_give_constant_hidden_layer():
    # W1 = 0: h = tanh(b1) for every row, y = W2 tanh(b1) + b2
    p, X, T, kw = tiny(1)
    W1, b1, W2, b2 = mlp.unpack(p, **kw)
    W1[:] = 0.0
    Hh, Y = mlp.forward(p, X, **kw)
    expect = W2 @ np.tanh(b1) + b2
    assert np.allclose(Hh, np.tanh(b1)[None, :], atol=0, rtol=1e-15)
    assert np.allclose(Y, expect[None, :], atol=1e-15, rtol=1e-14)
    # and dL/dW1 = 0 only where x is zero: with X = 0 the W1 gradient vanishes
    g = mlp.loss_grad(p, np.zeros_like(X), T, **kw)
    gW1, _, _, _ = mlp.unpack(g, **kw)
    assert np.all(gW1 == 0.0)


def test_output_bias_gradient_is_mean_residual():
    # dL/db2 = mean_b (y_b - t_b)
    p, X, T, kw = tiny(2)
    _, Y = mlp.forward(p, X, **kw)
    g = mlp.loss_grad(p, X, T, **kw)
    _, _, _, gb2 = mlp.unpack(g, **kw)
    assert np.allclose(gb2, (Y - T).mean(axis=0), atol=1e-15)


def test_perfect_fit_has_zero_loss_and_gradient():
    p, X, _, kw = tiny(3)
    _, Y = mlp.forward(p, X, **kw)
    assert mlp.loss(p, X, Y, **kw) == 0.0
    assert np.all(mlp.loss_grad(p, X, Y, **kw) == 0.0)


def test_first_adam_step_moves_by_lr_times_sign():
    # t = 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps)
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-2, 1e-8
    p1, m, v = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), atol=1e-15, rtol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_steps_stay_at_lr():
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -3.0])
    m = v = np.zeros(2)
    for t in range(1, 6):
        p_new, m, v = mlp.adam_step(p, g, m, v, t, 0.1, eps=0.0)
        assert np.allclose(p - p_new, 0.1 * np.sign(g), atol=1e-14)
        p = p_new
