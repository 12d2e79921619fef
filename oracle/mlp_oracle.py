"""FP64 reference of the surrogate network: a multilayer perceptron with SiLU
between layers, squared-error loss on standardised targets, its gradient by
the chain rule, and Adam.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark use it to check the GPU
network; the GPU library never does.

Conventions (those of the library's flat parameter vector): for each layer in
turn, W [out][in] row-major then b [out].  Activations: h_0 = standardised
input, z_l = h_{l-1} W_l^T + b_l, h_l = silu(z_l) = z_l * sigmoid(z_l) for the
hidden layers, yhat = z_L for the last.  Loss = mean over rows and outputs of
(yhat - (y - y_mean) / y_std)^2.

Adam is the published method of Kingma and Ba (ICLR 2015, Algorithm 1): with
gradient g_t, m_t = b1 m_{t-1} + (1 - b1) g_t, v_t = b2 v_{t-1} + (1 - b2) g_t^2,
theta_t = theta_{t-1} - lr * (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def layer_shapes(n_in, n_hidden, n_hidden_layers, n_out):
    dims = [n_in] + [n_hidden] * n_hidden_layers + [n_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]   # (out, in)


def param_count(shapes):
    return sum(o * i + o for o, i in shapes)


def unflatten(p, shapes):
    """Flat vector -> list of (W [out][in], b [out]) views (FP64 copies)."""
    p = np.asarray(p, dtype=np.float64)
    out, k = [], 0
    for o, i in shapes:
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.size
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def standardise(x, mean, std):
    std = np.where(np.asarray(std, np.float64) > 1e-12, std, 1.0)
    return (np.asarray(x, np.float64) - mean) / std


def forward(p, shapes, x_n):
    """Standardised inputs x_n [B][n_in] -> (yhat [B][n_out], cache)."""
    layers = unflatten(p, shapes)
    h = np.asarray(x_n, np.float64)
    zs, hs = [], [h]
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if l + 1 < len(layers) else z
        hs.append(h)
    return h, (zs, hs)


def predict(p, shapes, x, x_mean, x_std, y_mean, y_std):
    """Raw inputs -> raw outputs."""
    yhat, _ = forward(p, shapes, standardise(x, x_mean, x_std))
    y_std = np.where(np.asarray(y_std, np.float64) > 1e-12, y_std, 1.0)
    return yhat * y_std + y_mean


def loss_and_grad(p, shapes, x_n, y_n):
    """Mean squared error and its gradient (flat order) by the chain rule."""
    layers = unflatten(p, shapes)
    yhat, (zs, hs) = forward(p, shapes, x_n)
    B, n_out = yhat.shape
    e = yhat - y_n
    loss = float(np.mean(e * e))
    d = 2.0 * e / (B * n_out)                     # dL/dz_L
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (d.T @ hs[l], d.sum(axis=0))    # dL/dW_l, dL/db_l
        if l > 0:
            d = (d @ W) * silu_grad(zs[l - 1])
    return loss, flatten(grads)


def loss_only(p, shapes, x_n, y_n):
    yhat, _ = forward(p, shapes, x_n)
    return float(np.mean((yhat - y_n) ** 2))


class Adam:
    def __init__(self, n, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, p, g, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - lr * mh / (np.sqrt(vh) + self.eps)


def init_uniform(shapes, rng):
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases."""
    parts = []
    for o, i in shapes:
        bnd = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-bnd, bnd, o * i))
        parts.append(rng.uniform(-bnd, bnd, o))
    return np.concatenate(parts)


def column_stats(x):
    """Column means and population standard deviations in FP64."""
    x = np.asarray(x, np.float64)
    m = x.mean(axis=0)
    return m, np.sqrt(((x - m) ** 2).mean(axis=0))
