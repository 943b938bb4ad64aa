"""Cost-model network oracle -- test infrastructure only.

The learned cost model is not part of the paper: it stands in for the
hand-chosen efficiency parameters {eps_s} and recursion depth of Section 5
(the eps study) and for the nonzero count used as the load m in Sections
4.3-4.4.  Its definition is the textbook one, written out in float64:

    z1 = W1 x + b1,  h1 = relu(z1)          W1: 64 x 12
    z2 = W2 h1 + b2, h2 = relu(z2)          W2: 64 x 64
    f  = w3 . h2 + b3                       w3: 64

    L = (1/n) sum_s (f(x_s) - t_s)^2        (mean squared error)

The gradient is the chain rule taken by hand (relu'(z) = 1 for z > 0, else
0).  ``adam_step`` is the update of Kingma and Ba, "Adam: A Method for
Stochastic Optimization" (ICLR 2015, Algorithm 1), with bias correction.

Parameters travel as one flat vector in this order: W1 (row-major, output
by input), b1, W2 (row-major), b2, w3, b3 -- 5057 numbers.
"""
from __future__ import annotations

import numpy as np

N_IN = 12
N_HID = 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)), ("w3", (N_HID,)),
         ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    """Views of the flat parameter vector, in the order of SIZES."""
    theta = np.asarray(theta, dtype=np.float64)
    out, at = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[at:at + k].reshape(shape)
        at += k
    assert at == theta.size == N_PARAMS
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(seed):
    """He-style random initialisation (a starting point for tests and training)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2.0 / N_IN), (N_HID, N_IN)), "b1": np.zeros(N_HID),
         "W2": rng.normal(0, np.sqrt(2.0 / N_HID), (N_HID, N_HID)), "b2": np.zeros(N_HID),
         "w3": rng.normal(0, np.sqrt(1.0 / N_HID), N_HID), "b3": np.zeros(1)}
    return pack(p)


def forward(theta, X):
    """f(x_s) for every row x_s of X (n x 12)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    return h2 @ p["w3"] + p["b3"][0]


def loss_and_grad(theta, X, t):
    """Mean squared error and its gradient with respect to theta."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    f = h2 @ p["w3"] + p["b3"][0]
    r = f - t
    loss = float(np.mean(r * r))
    g = 2.0 * r / n                       # dL/df per sample
    d_w3 = h2.T @ g
    d_b3 = np.array([g.sum()])
    dz2 = np.outer(g, p["w3"]) * (z2 > 0)  # n x 64
    d_W2 = dz2.T @ h1
    d_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * (z1 > 0)       # n x 64
    d_W1 = dz1.T @ X
    d_b1 = dz1.sum(axis=0)
    grad = pack({"W1": d_W1, "b1": d_b1, "W2": d_W2, "b2": d_b2, "w3": d_w3, "b3": d_b3})
    return loss, grad


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
