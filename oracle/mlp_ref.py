"""FP64 reference of the learned QP-root seed (test infrastructure only).

A fully connected network 8 -> 64 -> 64 -> 1 with tanh on both hidden layers
and a linear output, trained with the mean squared error and Adam.  It is not
part of the paper: it predicts the quasiparticle shift from a handful of
self-energy samples so that the root search starts close to the root.

Parameter vector layout (4801 entries, the same order as the library's):
W1 [64, 8], b1 [64], W2 [64, 64], b2 [64], W3 [1, 64], b3 [1], each row-major.

Pins: central finite differences of the loss (gradients), the first Adam step
moving every parameter by -lr * sign(g) (the bias-corrected ratio is g/|g|),
and a network with only the output bias non-zero (closed-form loss/gradient).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H1, N_H2 = 8, 64, 64
SHAPES = [("W1", (N_H1, N_IN)), ("b1", (N_H1,)), ("W2", (N_H2, N_H1)), ("b2", (N_H2,)),
          ("W3", (1, N_H2)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta: np.ndarray):
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts)


def forward(theta: np.ndarray, x: np.ndarray):
    """y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 for each row of x [n, 8]."""
    p = unpack(theta)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y[:, 0], (h1, h2)


def loss_and_grad(theta: np.ndarray, x: np.ndarray, t: np.ndarray):
    """L = mean (y - t)^2 and dL/dtheta by backpropagation (chain rule)."""
    p = unpack(theta)
    n = x.shape[0]
    y, (h1, h2) = forward(theta, x)
    r = y - t
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]                 # [n, 1]
    g_w3 = dy.T @ h2
    g_b3 = dy.sum(axis=0)
    dz2 = (dy @ p["W3"]) * (1.0 - h2 * h2)      # [n, 64]
    g_w2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (1.0 - h1 * h1)
    g_w1 = dz1.T @ x
    g_b1 = dz1.sum(axis=0)
    grad = np.concatenate([g_w1.ravel(), g_b1, g_w2.ravel(), g_b2, g_w3.ravel(), g_b3])
    return loss, grad


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba, 2015), step number t >= 1.  In place."""
    m *= beta1
    m += (1.0 - beta1) * grad
    v *= beta2
    v += (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta -= lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
