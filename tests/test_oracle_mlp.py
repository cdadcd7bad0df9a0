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


def test_forward_hand_evaluated_network():
    """A network with non-zero weights whose pre-activations are logarithms:
    tanh(ln a) = (a^2 - 1) / (a^2 + 1), so every hidden value and the output
    are known fractions.  A missing or misplaced tanh, a transposed weight
    matrix or a dropped bias changes the output."""
    rng = np.random.default_rng(8)
    x = rng.standard_normal(M.N_IN)
    a1 = rng.choice([2.0, 3.0, 0.5, 1.5, 4.0, 0.25], M.N_H1)
    a2 = rng.choice([2.0, 3.0, 0.5, 1.5, 4.0, 0.25], M.N_H2)
    h1 = (a1 ** 2 - 1.0) / (a1 ** 2 + 1.0)
    h2 = (a2 ** 2 - 1.0) / (a2 ** 2 + 1.0)
    w1 = rng.standard_normal((M.N_H1, M.N_IN))
    w2 = 0.3 * rng.standard_normal((M.N_H2, M.N_H1))
    w3 = rng.standard_normal((1, M.N_H2))
    b1 = np.log(a1) - w1 @ x           # first pre-activations = ln a1
    b2 = np.log(a2) - w2 @ h1          # second pre-activations = ln a2
    b3 = np.array([0.25])
    theta = np.concatenate([w1.ravel(), b1, w2.ravel(), b2, w3.ravel(), b3])
    y, (g1, g2) = M.forward(theta, np.stack([x, x, x]))
    np.testing.assert_allclose(g1, np.broadcast_to(h1, g1.shape), rtol=0, atol=1e-14)
    np.testing.assert_allclose(g2, np.broadcast_to(h2, g2.shape), rtol=0, atol=1e-13)
    expect = float(w3[0] @ h2) + 0.25
    np.testing.assert_allclose(y, [expect] * 3, rtol=1e-13, atol=1e-13)
