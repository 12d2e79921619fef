"""Pins of the FP64 network oracle against things it does not compute itself:
finite differences, a library autograd, Adam's closed forms, SiLU identities."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M

SHAPES = M.layer_shapes(7, 12, 3, 5)


def _problem(seed=0, B=9):
    rng = np.random.default_rng(seed)
    p = M.init_uniform(SHAPES, rng)
    x = rng.normal(size=(B, 7))
    y = rng.normal(size=(B, 5))
    return p, x, y


def test_silu_identities():
    z = np.array([0.0, 40.0, -40.0, 1.0])
    s = M.silu(z)
    assert s[0] == 0.0 and abs(s[1] - 40.0) < 1e-12 and abs(s[2]) < 1e-15
    assert abs(s[3] - 1.0 / (1.0 + np.exp(-1.0))) < 1e-16
    g = M.silu_grad(np.array([0.0, 60.0, -60.0]))
    assert g[0] == 0.5 and abs(g[1] - 1.0) < 1e-12 and abs(g[2]) < 1e-12


def test_gradient_matches_central_differences():
    p, x, y = _problem()
    _, g = M.loss_and_grad(p, SHAPES, x, y)
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (M.loss_only(p + e, SHAPES, x, y) - M.loss_only(p - e, SHAPES, x, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-8 + 1e-6 * abs(fd), (k, fd, g[k])


def test_forward_and_gradient_match_torch_autograd():
    p, x, y = _problem(3, B=17)
    loss, g = M.loss_and_grad(p, SHAPES, x, y)
    tp = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    h = torch.tensor(x)
    k = 0
    for l, (o, i) in enumerate(SHAPES):
        W = tp[k:k + o * i].view(o, i)
        k += o * i
        b = tp[k:k + o]
        k += o
        h = torch.nn.functional.linear(h, W, b)
        if l + 1 < len(SHAPES):
            h = torch.nn.functional.silu(h)
    tl = torch.nn.functional.mse_loss(h, torch.tensor(y))
    tl.backward()
    assert abs(tl.item() - loss) < 1e-14
    np.testing.assert_allclose(g, tp.grad.numpy(), rtol=1e-10, atol=1e-15)
    yhat, _ = M.forward(p, SHAPES, x)
    np.testing.assert_allclose(yhat, h.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_flat_order_is_weights_then_bias_per_layer():
    shapes = M.layer_shapes(2, 3, 1, 1)
    assert M.param_count(shapes) == 3 * 2 + 3 + 1 * 3 + 1
    p = np.arange(13, dtype=float)
    (W0, b0), (W1, b1) = M.unflatten(p, shapes)
    np.testing.assert_array_equal(W0, [[0, 1], [2, 3], [4, 5]])
    np.testing.assert_array_equal(b0, [6, 7, 8])
    np.testing.assert_array_equal(W1, [[9, 10, 11]])
    np.testing.assert_array_equal(b1, [12])
    np.testing.assert_array_equal(M.flatten(M.unflatten(p, shapes)), p)


def test_adam_first_step_and_constant_gradient_closed_forms():
    g = np.array([3.0, -2e-3, 0.0, 1e-9])
    lr = 0.01
    opt = M.Adam(4, lr)
    p0 = np.zeros(4)
    p1 = opt.step(p0, g)
    # step 1: bias-corrected m = g, v = g^2
    np.testing.assert_allclose(p1, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # constant gradient: every step moves by the same amount
    p = p1
    for t in range(2, 50):
        q = opt.step(p, g)
        np.testing.assert_allclose(q - p, p1 - p0, rtol=1e-9, atol=1e-18)
        p = q


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p = rng.normal(size=20)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt_t = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    opt = M.Adam(20, 3e-3)
    for _ in range(25):
        g = rng.normal(size=20)
        p = opt.step(p, g)
        tp.grad = torch.tensor(g)
        opt_t.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_standardise_and_column_stats():
    rng = np.random.default_rng(2)
    x = rng.normal(3.0, 2.0, size=(1000, 4))
    x[:, 2] = 7.0                               # a constant column
    m, s = M.column_stats(x)
    np.testing.assert_allclose(m, x.mean(0), rtol=1e-14)
    np.testing.assert_allclose(s, x.std(0), rtol=1e-12, atol=1e-15)
    xn = M.standardise(x, m, s)
    np.testing.assert_allclose(xn[:, [0, 1, 3]].mean(0), 0, atol=1e-12)
    np.testing.assert_allclose(xn[:, [0, 1, 3]].std(0), 1, rtol=1e-12)
    np.testing.assert_allclose(xn[:, 2], 0.0, atol=1e-12)   # std 0 -> divided by 1


def test_predict_inverts_target_standardisation():
    """With zero last-layer weights the prediction is b_L * y_std + y_mean."""
    p, x, _ = _problem(7)
    layers = M.unflatten(p, SHAPES)
    layers[-1] = (np.zeros_like(layers[-1][0]), np.array([0.5, -1, 0, 2, 3.0]))
    q = M.flatten(layers)
    ym, ys = np.arange(5.0), np.array([1, 2, 0, 4, 5.0])
    out = M.predict(q, SHAPES, x, np.zeros(7), np.ones(7), ym, ys)
    np.testing.assert_allclose(out, np.tile([0.5, -1, 2, 11, 19.0], (x.shape[0], 1)), atol=1e-14)
