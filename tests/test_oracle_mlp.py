"""Pins of the reference MLP (forward, back-propagation, Adam) against finite differences,
closed forms and the Adam update formula."""
import numpy as np

from oracle import mlp
from oracle.lowprec import to_bf16


def _net(dims, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((o, i)) / np.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(dims[:-1], dims[1:])]


def test_forward_closed_form():
    """One hidden unit: y = 3 tanh(2 x + 0.5) - 1."""
    params = [(np.array([[2.0]]), np.array([0.5])), (np.array([[3.0]]), np.array([-1.0]))]
    x = np.array([[-1.0], [0.0], [0.7]])
    y, _ = mlp.forward(params, x)
    assert np.allclose(y[:, 0], 3.0 * np.tanh(2.0 * x[:, 0] + 0.5) - 1.0, rtol=0, atol=1e-15)


def test_gradients_match_central_differences():
    dims = [3, 7, 5, 2]
    params = _net(dims, 1)
    rng = np.random.default_rng(2)
    X, T = rng.standard_normal((6, 3)), rng.standard_normal((6, 2))

    def loss(vec):
        y, _ = mlp.forward(mlp.unflatten(vec, dims), X)
        return mlp.mse(y, T)[0]

    y, acts = mlp.forward(params, X)
    _, dy = mlp.mse(y, T)
    g = mlp.flatten([(gw, gb) for gw, gb in mlp.backward(params, acts, dy)])
    v = mlp.flatten(params)
    h = 1e-6
    fd = np.array([(loss(v + h * e) - loss(v - h * e)) / (2 * h) for e in np.eye(v.size)])
    assert np.abs(fd - g).max() <= 1e-8 * max(1.0, np.abs(g).max())


def test_adam_first_step_is_sign_step():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so every parameter moves by
    lr g / (|g| + eps)."""
    dims = [2, 3, 1]
    params = _net(dims, 3)
    grads = _net(dims, 4)
    new, (t, m, v) = mlp.adam(params, grads, None, lr=1e-3)
    assert t == 1
    for (W, b), (gW, gb), (W2, b2) in zip(params, grads, new):
        assert np.allclose(W - W2, 1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-12, atol=0)
        assert np.allclose(b - b2, 1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=0)
    # second step with the same gradient: moments stay aligned, step size unchanged
    new2, _ = mlp.adam(new, grads, (t, m, v), lr=1e-3)
    for (W, _), (W2, _), (gW, _) in zip(new, new2, grads):
        assert np.allclose(W - W2, 1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-9, atol=0)


def test_bf16_mode_rounds_where_stated():
    dims = [4, 8, 3]
    params = _net(dims, 5)
    X = np.random.default_rng(6).standard_normal((5, 4))
    y, acts = mlp.forward(params, X, bf16=True)
    for a in acts:
        assert np.array_equal(to_bf16(a), a)
    W1, b1 = params[0]
    a1 = to_bf16(np.tanh(to_bf16(X) @ to_bf16(W1).T + b1))
    assert np.array_equal(acts[1], a1)
    W2, b2 = params[1]
    assert np.allclose(y, a1 @ to_bf16(W2).T + b2, rtol=1e-15, atol=1e-15)
    # back-propagated gradients are bfloat16 values; db sums them
    _, dy = mlp.mse(y, np.zeros_like(y))
    grads = mlp.backward(params, acts, dy, bf16=True)
    g2 = to_bf16(dy)
    assert np.allclose(grads[1][1], g2.sum(axis=0), rtol=1e-15, atol=0)
    g1 = to_bf16((g2 @ to_bf16(W2)) * (1.0 - a1 * a1))
    assert np.allclose(grads[0][0], g1.T @ acts[0], rtol=1e-14, atol=0)


def test_training_reduces_loss():
    dims = [1, 16, 1]
    params = _net(dims, 7)
    x = np.linspace(-2, 2, 64)[:, None]
    t = np.sin(2 * x)
    state = None
    l0 = mlp.mse(mlp.forward(params, x)[0], t)[0]
    for _ in range(400):
        y, acts = mlp.forward(params, x)
        _, dy = mlp.mse(y, t)
        params, state = mlp.adam(params, mlp.backward(params, acts, dy), state, lr=1e-2)
    l1 = mlp.mse(mlp.forward(params, x)[0], t)[0]
    assert l1 < 0.05 * l0


def test_modulated_output_gradients():
    """Output linear in per-sample weights f: y[k] = sum_i f_i z[i K + k]; gradients against
    central differences, and the output for one-hot f picks the matching slice of z."""
    dims = [4, 9, 6]          # n_mod = 3, K = 2
    params = _net(dims, 8)
    rng = np.random.default_rng(9)
    X, F, T = rng.standard_normal((5, 4)), rng.standard_normal((5, 3)), rng.standard_normal((5, 2))

    def loss(vec):
        z, _ = mlp.forward(mlp.unflatten(vec, dims), X)
        return mlp.mse(mlp.modulate(z, F), T)[0]

    z, acts = mlp.forward(params, X)
    _, dy = mlp.mse(mlp.modulate(z, F), T)
    g = mlp.flatten(mlp.backward(params, acts, dy, f=F))
    v = mlp.flatten(params)
    h = 1e-6
    fd = np.array([(loss(v + h * e) - loss(v - h * e)) / (2 * h) for e in np.eye(v.size)])
    assert np.abs(fd - g).max() <= 1e-8 * max(1.0, np.abs(g).max())
    onehot = np.zeros((5, 3))
    onehot[:, 1] = 1.0
    assert np.array_equal(mlp.modulate(z, onehot), z[:, 2:4])
