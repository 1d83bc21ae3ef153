"""Pins of the FP64 proposal-network oracle: central finite differences of the
loss, closed-form special cases, the first Adam step, Adam over five steps
of a constant gradient and two steps worked by hand."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.n_params() == 6337
    p = mlp.init_params(0)
    assert mlp.flatten(p).size == 6337
    q = mlp.unflatten(mlp.flatten(p))
    for k, _ in mlp.SHAPES:
        np.testing.assert_array_equal(p[k], q[k])


def test_zero_network_loss_is_log2():
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    x = np.random.default_rng(0).standard_normal((16, 32))
    y = (np.arange(16) % 2).astype(float)
    assert mlp.loss(p, x, y) == pytest.approx(math.log(2.0), abs=1e-15)
    f = mlp.forward(p, x)
    np.testing.assert_allclose(f["score"], 0.5, atol=0)


def test_bias_only_logistic_regression():
    """With all weights zero the logit is b3 for every row: the loss is the
    Bernoulli cross-entropy of sigmoid(b3), with derivative sigmoid(b3) - mean(y)."""
    p = {k: np.zeros(s) for k, s in mlp.SHAPES}
    p["b3"] = np.array([0.3])
    x = np.random.default_rng(1).standard_normal((10, 32))
    y = np.array([1, 1, 1, 0, 1, 0, 1, 1, 0, 1], dtype=float)
    s = 1 / (1 + math.exp(-0.3))
    want = -(y.mean() * math.log(s) + (1 - y.mean()) * math.log(1 - s))
    assert mlp.loss(p, x, y) == pytest.approx(want, abs=1e-14)
    g = mlp.backward(p, x, y)
    assert g["b3"][0] == pytest.approx(s - y.mean(), abs=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    p = mlp.init_params(seed)
    g = np.random.default_rng(seed + 10)
    x = g.standard_normal((8, 32))
    y = (g.random(8) < 0.5).astype(float)
    grad = mlp.flatten(mlp.backward(p, x, y))
    vec = mlp.flatten(p)
    idx = g.choice(vec.size, 200, replace=False)
    h = 1e-6
    for i in idx:
        vp, vm = vec.copy(), vec.copy()
        vp[i] += h
        vm[i] -= h
        fd = (mlp.loss(mlp.unflatten(vp), x, y) - mlp.loss(mlp.unflatten(vm), x, y)) / (2 * h)
        assert abs(fd - grad[i]) < 1e-8 + 1e-5 * abs(fd), (i, fd, grad[i])


def test_first_adam_step_moves_by_lr():
    """Bias correction makes the first step lr * g/(|g| + eps') = lr * sign(g)."""
    p = mlp.init_params(3)
    x = np.random.default_rng(4).standard_normal((32, 32))
    y = (np.arange(32) % 3 == 0).astype(float)
    g = mlp.backward(p, x, y)
    m = {k: np.zeros(s) for k, s in mlp.SHAPES}
    v = {k: np.zeros(s) for k, s in mlp.SHAPES}
    before = {k: p[k].copy() for k in p}
    mlp.adam_step(p, g, m, v, step=1, lr=1e-3, eps=0.0)
    for k, _ in mlp.SHAPES:
        nz = g[k] != 0
        np.testing.assert_allclose((before[k] - p[k])[nz], 1e-3 * np.sign(g[k][nz]), rtol=1e-9)


def test_training_reduces_loss_on_separable_labels():
    g = np.random.default_rng(5)
    x = g.standard_normal((512, 32))
    y = (x[:, 0] + 0.5 * x[:, 3] > 0).astype(float)
    p = mlp.init_params(6)
    m = {k: np.zeros(s) for k, s in mlp.SHAPES}
    v = {k: np.zeros(s) for k, s in mlp.SHAPES}
    l0 = mlp.loss(p, x, y)
    for step in range(1, 201):
        mlp.adam_step(p, mlp.backward(p, x, y), m, v, step, lr=1e-2)
    assert mlp.loss(p, x, y) < 0.3 * l0


def test_adam_constant_gradient_moves_lr_each_step():
    """With the same gradient every step the bias-corrected moments equal g and
    g^2 exactly (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each of the
    steps moves every parameter by lr * sign(g) when eps = 0."""
    p = mlp.init_params(7)
    x = np.random.default_rng(8).standard_normal((16, 32))
    y = (np.arange(16) % 2).astype(float)
    g = mlp.backward(p, x, y)
    m = {k: np.zeros(s) for k, s in mlp.SHAPES}
    v = {k: np.zeros(s) for k, s in mlp.SHAPES}
    for step in range(1, 6):
        before = {k: p[k].copy() for k in p}
        mlp.adam_step(p, g, m, v, step=step, lr=1e-3, eps=0.0)
        for k, _ in mlp.SHAPES:
            nz = g[k] != 0
            np.testing.assert_allclose((before[k] - p[k])[nz], 1e-3 * np.sign(g[k][nz]),
                                       rtol=1e-9)


def test_adam_two_steps_by_hand():
    """Every parameter 0.5, gradient 1 then -2, lr 0.1, b1 0.9, b2 0.999, eps 0.
    Step 1: m = 0.1, v = 0.001, corrected 1 and 1, so 0.5 -> 0.4.
    Step 2: m = 0.09 - 0.2 = -0.11, v = 0.000999 + 0.004 = 0.004999;
    corrected m = -0.11/0.19 = -11/19, v = 0.004999/0.001999 = 4999/1999;
    0.4 -> 0.4 + (11/190) * sqrt(1999/4999) = 0.43661035270358456."""
    p = {k: np.full(s, 0.5) for k, s in mlp.SHAPES}
    m = {k: np.zeros(s) for k, s in mlp.SHAPES}
    v = {k: np.zeros(s) for k, s in mlp.SHAPES}
    mlp.adam_step(p, {k: np.full(s, 1.0) for k, s in mlp.SHAPES}, m, v, 1,
                  lr=0.1, eps=0.0)
    for k, _ in mlp.SHAPES:
        np.testing.assert_allclose(p[k], 0.4, rtol=1e-14)
    mlp.adam_step(p, {k: np.full(s, -2.0) for k, s in mlp.SHAPES}, m, v, 2,
                  lr=0.1, eps=0.0)
    for k, _ in mlp.SHAPES:
        np.testing.assert_allclose(p[k], 0.43661035270358456, rtol=1e-14)
