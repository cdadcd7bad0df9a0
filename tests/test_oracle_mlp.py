"""Pins of the FP64 MLP reference (finite differences, closed forms)."""
import numpy as np
import pytest

from oracle import mlp_ref as M


def data(n=37, seed=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, M.N_IN))
    t = rng.standard_normal(n) * 0.5
    return x, t


def test_param_count():
    assert M.N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4801


def test_gradient_central_differences():
    x, t = data()
    theta = M.init_params(1)
    theta[M.N_PARAMS - 1] = 0.1
    _, g = M.loss_and_grad(theta, x, t)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(M.N_PARAMS, 60, replace=False),
                          [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4799, 4800]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss_and_grad(tp, x, t)[0] - M.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_output_bias_only_network():
    x, t = data()
    theta = np.zeros(M.N_PARAMS)
    theta[-1] = 0.7
    loss, g = M.loss_and_grad(theta, x, t)
    assert loss == pytest.approx(np.mean((0.7 - t) ** 2), rel=1e-14)
    assert g[-1] == pytest.approx(2 * np.mean(0.7 - t), rel=1e-14)
    # with all weights zero, every other gradient vanishes except dL/dW3 = 0 too
    assert np.all(g[:-1] == 0.0)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    grad = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    th0 = theta.copy()
    M.adam_step(theta, grad, m, v, 1, lr=1e-2, eps=0.0)
    np.testing.assert_allclose(theta - th0, -1e-2 * np.sign(grad), rtol=1e-12)


def test_adam_minimises_quadratic():
    theta = np.array([3.0, -2.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 3001):
        M.adam_step(theta, 2 * theta, m, v, t, lr=0.01)
    assert np.max(np.abs(theta)) < 1e-2
