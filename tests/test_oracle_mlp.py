"""Pins of the float64 reference network (oracle/mlp.py): finite differences,
a closed form for the all-active network, the first Adam step, and a short
training run that must reduce the loss on a smooth target."""
import numpy as np
import pytest

from oracle import mlp


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(n, mlp.NI))
    T = np.stack([np.sin(X[:, 0]) + X[:, 1] * X[:, 2], X[:, 0] - 0.5 * X[:, 1] ** 2], 1)
    return X, T


def _loss(theta, X, T):
    Y, _ = mlp.forward(theta, X)
    return mlp.mse(Y, T)[0]


def test_nparam():
    assert mlp.NPARAM == 64 * 3 + 64 + 2 * (64 * 64 + 64) + 2 * 64 + 2


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_central_differences(seed):
    X, T = _data(7, seed)
    theta = mlp.init(seed)
    theta[mlp.NPARAM - 2:] = 0.3               # nonzero output bias
    Y, acts = mlp.forward(theta, X)
    _, dY = mlp.mse(Y, T)
    g = mlp.backward(theta, acts, dY)
    rng = np.random.default_rng(100 + seed)
    # every bias of every layer plus a random sample of weights
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    idx = set(rng.choice(mlp.NPARAM, 120, replace=False).tolist())
    for k, (name, _) in enumerate(mlp.SHAPES):
        if name.startswith("b"):
            idx.update(range(offs[k], offs[k + 1]))
    h = 1e-6
    for i in sorted(idx):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (_loss(tp, X, T) - _loss(tm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, g[i])


def test_all_active_network_is_affine():
    """With positive weights, nonnegative inputs and positive biases every
    ReLU is in its linear part, so the network is the product of its affine
    maps."""
    rng = np.random.default_rng(3)
    parts = {}
    for name, shp in mlp.SHAPES:
        parts[name] = rng.uniform(0.01, 0.1, size=shp)
    theta = mlp.pack(parts)
    X = rng.uniform(0, 1, size=(5, mlp.NI))
    Y, _ = mlp.forward(theta, X)
    A = parts["W4"] @ parts["W3"] @ parts["W2"] @ parts["W1"]
    c = parts["W4"] @ (parts["W3"] @ (parts["W2"] @ parts["b1"] + parts["b2"]) + parts["b3"]) + parts["b4"]
    np.testing.assert_allclose(Y, X @ A.T + c, rtol=1e-12)


def test_dead_network_outputs_bias():
    """All first-layer pre-activations negative: every hidden unit is zero and
    the output is b4 regardless of the input; all gradients but b4's vanish."""
    parts = {name: np.zeros(shp) for name, shp in mlp.SHAPES}
    parts["b1"][:] = -1.0
    parts["b4"][:] = [2.0, -3.0]
    parts["W2"][:] = 1.0
    theta = mlp.pack(parts)
    X = np.random.default_rng(4).uniform(-0.5, 0.5, size=(6, 3))
    Y, acts = mlp.forward(theta, X)
    np.testing.assert_array_equal(Y, np.tile([2.0, -3.0], (6, 1)))
    g = mlp.backward(theta, acts, np.ones_like(Y))
    np.testing.assert_array_equal(g[:-2], 0.0)
    np.testing.assert_array_equal(g[-2:], [6.0, 6.0])


def test_mse_gradient():
    rng = np.random.default_rng(5)
    Y, T = rng.normal(size=(4, 2)), rng.normal(size=(4, 2))
    L, dY = mlp.mse(Y, T)
    assert L == pytest.approx(np.sum((Y - T) ** 2) / 8)
    h = 1e-6
    for i in range(4):
        for j in range(2):
            Yp = Y.copy(); Yp[i, j] += h
            Ym = Y.copy(); Ym[i, j] -= h
            assert (mlp.mse(Yp, T)[0] - mlp.mse(Ym, T)[0]) / (2 * h) == pytest.approx(dY[i, j], rel=1e-6)


def test_first_adam_step_is_lr_times_sign():
    rng = np.random.default_rng(6)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    g[7] = 0.0
    t1, m, v = mlp.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    step = theta - t1
    np.testing.assert_allclose(step[g != 0], 1e-3 * np.sign(g[g != 0]), rtol=1e-6)
    assert step[7] == 0.0
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    X, T = _data(128, 7)
    theta, hist = mlp.train(mlp.init(7), X, T, steps=300, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0]
