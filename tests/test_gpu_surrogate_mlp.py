"""GPU parity of the surrogate network's kernels (forward, loss, gradient, Adam,
column statistics) against the FP64 network oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

SHAPE = dict(n_in=293, n_hidden=256, n_hidden_layers=3, n_out=49)


def _torch():
    import torch
    return torch


def say(msg):
    print(msg, flush=True)


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) & 0xFFFF0000
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def _make(precision, max_batch=1024, seed=11, training=True):
    from paper_2411_05799_amd import native as N
    return N.Surrogate(max_batch=max_batch, precision=precision, training=training, seed=seed,
                       **SHAPE)


def _data(rng, rows, bf16=False):
    x = rng.normal(0.3, 1.7, size=(rows, SHAPE["n_in"]))
    y = rng.normal(-0.2, 0.8, size=(rows, SHAPE["n_out"]))
    xm, xs = x.mean(0), x.std(0)
    ym, ys = y.mean(0), y.std(0)
    if bf16:   # identity standardisation so that the BF16 operands are the inputs themselves
        x = bf16_round(x)
        xm, xs = np.zeros(SHAPE["n_in"]), np.ones(SHAPE["n_in"])
    return x.astype(np.float32), y.astype(np.float32), xm, xs, ym, ys


def _dev(a, dtype=None):
    torch = _torch()
    return torch.tensor(a, device="cuda", dtype=dtype)


def _shapes():
    return M.layer_shapes(SHAPE["n_in"], SHAPE["n_hidden"], SHAPE["n_hidden_layers"], SHAPE["n_out"])


def test_initial_params_are_uniform_in_fan_in_bounds():
    from paper_2411_05799_amd import native as N
    s = _make(N.SUR_FP32, max_batch=64)
    p = s.get_params().astype(np.float64)
    assert p.size == M.param_count(_shapes()) == 219441
    for (W, b), (o, i) in zip(M.unflatten(p, _shapes()), _shapes()):
        bnd = 1 / np.sqrt(i)
        assert np.abs(W).max() <= bnd and np.abs(b).max() <= bnd
        assert abs(W.std() - bnd / np.sqrt(3)) < 0.05 * bnd
    q = np.random.default_rng(0).normal(size=p.size).astype(np.float32)
    s.set_params(q)
    np.testing.assert_array_equal(s.get_params(), q)
    s.close()


@pytest.mark.parametrize("batch", [1, 37, 300, 1024])
def test_forward_fp32_matches_oracle(batch):
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(batch)
    x, y, xm, xs, ym, ys = _data(rng, 1500)
    s = _make(N.SUR_FP32)
    s.set_norm(xm, xs, ym, ys)
    p = s.get_params().astype(np.float64)
    rows = rng.choice(1500, batch, replace=False).astype(np.int32)
    out = torch.full((batch, 64), 7.0, device="cuda")
    s.forward(_dev(x), out[:, :49], rows=_dev(rows))
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = M.predict(p, _shapes(), x[rows].astype(np.float64), xm.astype(np.float32),
                    xs.astype(np.float32), ym.astype(np.float32), ys.astype(np.float32))
    err = np.abs(got[:, :49] - ref).max() / np.abs(ref).max()
    assert err <= 1e-5, err
    assert np.all(got[:, 49:] == 7.0)        # columns past n_out untouched
    s.close()


def abs_term_sums(p, x_n, y_n):
    """Per parameter, the sum of the absolute values of the terms whose sum is
    its gradient (flat order): |d_l|^T |h_{l-1}| for a weight block and the sum
    of |d_l| over rows for a bias, with the FP64 back-propagated d_l and
    activations h of the oracle's forward pass. A float32 sum of these terms
    is off by at most a small multiple of float32 rounding times this sum."""
    layers = M.unflatten(p, _shapes())
    yhat, (zs, hs) = M.forward(p, _shapes(), x_n)
    B, n_out = yhat.shape
    d = 2.0 * (yhat - y_n) / (B * n_out)
    out = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        out[l] = (np.abs(d).T @ np.abs(hs[l]), np.abs(d).sum(axis=0))
        if l > 0:
            d = (d @ W) * M.silu_grad(zs[l - 1])
    return M.flatten(out)


def _grad_case(precision, batch, seed):
    from paper_2411_05799_amd import native as N
    torch = _torch()
    bf16 = precision == N.SUR_BF16
    rng = np.random.default_rng(seed)
    x, y, xm, xs, ym, ys = _data(rng, batch, bf16=bf16)
    s = _make(precision)
    if bf16:
        s.set_params(bf16_round(s.get_params()))
    s.set_norm(xm, xs, ym, ys)
    p = s.get_params().astype(np.float64)
    loss = torch.zeros(1, device="cuda")
    g = torch.zeros(p.size, device="cuda")
    s.grad(_dev(x), _dev(y), loss=loss, grad=g)
    torch.cuda.synchronize()
    f32 = np.float32
    xn = M.standardise(x.astype(np.float64), xm.astype(f32), xs.astype(f32))
    yn = M.standardise(y.astype(np.float64), ym.astype(f32), ys.astype(f32))
    l_ref, g_ref = M.loss_and_grad(p, _shapes(), xn, yn)
    A = abs_term_sums(p, xn, yn)
    s.close()
    return float(loss.item()), l_ref, g.cpu().numpy().astype(np.float64), g_ref, A


def _blocks(v):
    return [(f"{n}{k}", a) for k, (W, b) in enumerate(M.unflatten(v, _shapes()))
            for n, a in (("W", W), ("b", b))]


@pytest.mark.parametrize("batch", [64, 200, 1024])
def test_gradient_fp32_matches_oracle(batch):
    """Every entry of every weight and bias gradient within 1e-5 of its own
    value plus 1e-5 of its sum of absolute terms (the rounding of a float32
    sum of terms of mixed signs scales with that sum, not with the sum's own
    value, which cancellation can make small); the loss, the whole gradient
    and each block's norm within 1e-5."""
    from paper_2411_05799_amd import native as N
    l, l_ref, g, g_ref, A = _grad_case(N.SUR_FP32, batch, 5 + batch)
    assert abs(l - l_ref) <= 1e-6 * l_ref
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    assert rel <= 1e-5, rel
    for (n, a), (_, r), (_, t) in zip(_blocks(g), _blocks(g_ref), _blocks(A)):
        assert np.linalg.norm(a - r) <= 1e-5 * np.linalg.norm(r), n
    ratio = {n: float((np.abs(a - r) / (np.abs(r) + t)).max())
             for (n, a), (_, r), (_, t) in zip(_blocks(g), _blocks(g_ref), _blocks(A))}
    say(f"fp32 gradient, batch {batch}: largest |g - g_ref| / (|g_ref| + sum|terms|) per block "
        + ", ".join(f"{n} {v:.1e}" for n, v in ratio.items()))
    for n, v in ratio.items():
        assert v <= 1e-5, (n, v)


def test_gradient_bf16_within_1e_2_of_oracle():
    """BF16 operands with FP32 accumulation: the loss and each block's norm
    within 1e-2, and every entry within 1e-2 of its own value plus its sum of
    absolute terms (activations are rounded to BF16, 2^-9 relative, between
    layers)."""
    from paper_2411_05799_amd import native as N
    l, l_ref, g, g_ref, A = _grad_case(N.SUR_BF16, 1000, 3)
    assert abs(l - l_ref) <= 1e-2 * l_ref
    for (n, a), (_, r) in zip(_blocks(g), _blocks(g_ref)):
        assert np.linalg.norm(a - r) <= 1e-2 * np.linalg.norm(r), n
    ratio = {n: float((np.abs(a - r) / (np.abs(r) + t)).max())
             for (n, a), (_, r), (_, t) in zip(_blocks(g), _blocks(g_ref), _blocks(A))}
    say("bf16 gradient: largest |g - g_ref| / (|g_ref| + sum|terms|) per block "
        + ", ".join(f"{n} {v:.1e}" for n, v in ratio.items()))
    for n, v in ratio.items():
        assert v <= 1e-2, (n, v)


def test_forward_bf16_within_1e_2_of_oracle():
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(8)
    x, y, xm, xs, ym, ys = _data(rng, 500, bf16=True)
    s = _make(N.SUR_BF16)
    s.set_params(bf16_round(s.get_params()))
    s.set_norm(xm, xs, ym, ys)
    p = s.get_params().astype(np.float64)
    out = torch.zeros((500, 49), device="cuda")
    s.forward(_dev(x), out)
    torch.cuda.synchronize()
    f32 = np.float32
    ref = M.predict(p, _shapes(), x.astype(np.float64), xm, xs, ym.astype(f32), ys.astype(f32))
    got = out.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-2 * np.linalg.norm(ref - ym.astype(f32))
    # every output against the spread of its column (the de-standardised scale)
    col = np.abs(ref - ym.astype(f32)).max(0)
    ew = float((np.abs(got - ref) / col[None, :]).max())
    say(f"bf16 forward: largest elementwise error / column scale {ew:.2e}")
    assert ew <= 1e-2, ew
    s.close()


def test_adam_step_fp32_matches_oracle():
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(21)
    x, y, xm, xs, ym, ys = _data(rng, 512)
    s = _make(N.SUR_FP32)
    s.set_norm(xm, xs, ym, ys)
    p = s.get_params().astype(np.float64)
    f32 = np.float32
    xn = M.standardise(x.astype(np.float64), xm.astype(f32), xs.astype(f32))
    yn = M.standardise(y.astype(np.float64), ym.astype(f32), ys.astype(f32))
    opt = M.Adam(p.size, 1e-3)
    lrs = [1e-3, 5e-4, 2e-4]
    xd, yd = _dev(x), _dev(y)
    for lr in lrs:
        _, g_ref = M.loss_and_grad(p, _shapes(), xn, yn)
        p_new = opt.step(p, g_ref, lr=lr)
        s.train_step(xd, yd, lr)
        got = s.get_params().astype(np.float64)
        # Adam's step is insensitive to gradient error except where |g| is near eps
        big = np.abs(g_ref) > 1e-4 * np.abs(g_ref).max()
        assert np.abs((got - p_new)[big]).max() <= 2e-3 * lr
        assert np.abs(got - p_new).max() <= 2.0 * lr + 1e-6
        p = got     # continue both from the GPU's parameters
    s.close()


def test_training_reduces_loss_and_is_deterministic():
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(4)
    n = 8192
    x = rng.normal(size=(n, SHAPE["n_in"])).astype(np.float32)
    A = rng.normal(size=(SHAPE["n_in"], SHAPE["n_out"])) / np.sqrt(SHAPE["n_in"])
    y = np.tanh(x @ A).astype(np.float32)
    xd, yd = _dev(x), _dev(y)
    xm, xs = norm_stats_host(x)
    ym, ys = norm_stats_host(y)
    losses, params = [], []
    for rep in range(2):
        s = _make(N.SUR_BF16, max_batch=1024, seed=3)
        s.set_norm(xm, xs, ym, ys)
        loss = torch.zeros(1, device="cuda")
        g = torch.Generator().manual_seed(0)
        hist = []
        for it in range(150):
            rows = torch.randint(0, n, (1024,), generator=g, dtype=torch.int32).cuda()
            s.train_step(xd, yd, 2e-3, loss=loss, rows=rows)
            hist.append(loss.item())
        losses.append(hist)
        params.append(s.get_params())
        s.close()
    assert np.mean(losses[0][-10:]) < 0.25 * np.mean(losses[0][:3]), (losses[0][:3], losses[0][-10:])
    np.testing.assert_array_equal(params[0], params[1])
    assert losses[0] == losses[1]


def norm_stats_host(a):
    m, s = M.column_stats(a)
    return m.astype(np.float32), s.astype(np.float32)


def test_norm_stats_match_numpy():
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(9)
    rows, ld, cols = 100003, 345, 342
    a = rng.normal(2.0, 3.0, size=(rows, ld)).astype(np.float32)
    a[:, 5] = 1.25
    m, s = N.norm_stats(_dev(a), cols=cols)
    mr, sr = M.column_stats(a[:, :cols].astype(np.float64))
    np.testing.assert_allclose(m.cpu().numpy(), mr, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(s.cpu().numpy(), sr, rtol=1e-6, atol=1e-7)
    assert s[5].item() == 0.0


def test_edge_cases_and_errors():
    from paper_2411_05799_amd import native as N
    torch = _torch()
    s = _make(N.SUR_BF16, max_batch=100, training=False)
    x = torch.zeros((200, SHAPE["n_in"]), device="cuda")
    out = torch.zeros((200, 49), device="cuda")
    s.forward(x, out, batch=0)                      # empty batch: no work
    with pytest.raises(N.NpxError):
        s.forward(x, out)                           # 200 > max_batch
    with pytest.raises(N.NpxError):
        s.grad(x[:10], out[:10])                    # no training buffers
    s.forward(x[:100], out[:100])                   # exactly max_batch
    torch.cuda.synchronize()
    assert torch.isfinite(out[:100]).all() and (out[100:] == 0).all()
    s.close()
    with pytest.raises(N.NpxError):
        N.Surrogate(n_in=3, n_hidden=8, n_hidden_layers=0, n_out=1, max_batch=4)


def test_training_noise_shifts_inputs_and_targets():
    """With training noise set, the gradient is the oracle's on inputs + noise
    and targets - noise in the same columns; inference ignores the noise."""
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(31)
    batch = 300
    x, y, xm, xs, ym, ys = _data(rng, batch)
    s = _make(N.SUR_FP32)
    s.set_norm(xm, xs, ym, ys)
    p = s.get_params().astype(np.float64)
    nz = (rng.normal(size=(batch, 11)) * 0.3).astype(np.float32)
    nz_d = _dev(nz)
    s.set_noise(nz_d, col0=2)
    loss = torch.zeros(1, device="cuda")
    g = torch.zeros(p.size, device="cuda")
    s.grad(_dev(x), _dev(y), loss=loss, grad=g)
    out = torch.zeros((batch, 49), device="cuda")
    s.forward(_dev(x), out)
    torch.cuda.synchronize()
    f32 = np.float32
    xn_in = x.astype(np.float64).copy()
    yn_in = y.astype(np.float64).copy()
    xn_in[:, 2:13] += nz
    yn_in[:, 2:13] -= nz
    xn = M.standardise(xn_in, xm.astype(f32), xs.astype(f32))
    yn = M.standardise(yn_in, ym.astype(f32), ys.astype(f32))
    l_ref, g_ref = M.loss_and_grad(p, _shapes(), xn, yn)
    assert abs(loss.item() - l_ref) <= 1e-6 * l_ref
    assert np.linalg.norm(g.cpu().numpy() - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    ref = M.predict(p, _shapes(), x.astype(np.float64), xm.astype(f32), xs.astype(f32),
                    ym.astype(f32), ys.astype(f32))
    got = out.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    with pytest.raises(N.NpxError):
        s.set_noise(_dev(np.zeros((batch, 60), np.float32)), col0=2)   # past the outputs
    s.set_noise(None)
    s.close()


@pytest.mark.parametrize("shape", [
    dict(n_in=293, n_hidden=256, n_hidden_layers=3, n_out=49),    # one fused launch
    dict(n_in=293, n_hidden=384, n_hidden_layers=4, n_out=49),    # fused, three blocks per wave
    dict(n_in=293, n_hidden=256, n_hidden_layers=3, n_out=100),   # layer by layer, 128x128 tiles
], ids=["fused256", "fused384", "tiled"])
def test_forward_bf16_large_batch_matches_oracle_on_sampled_rows(shape):
    """65,536 rows: the whole-network kernel (widths it takes) or the 128x128
    tiles of the layer-by-layer forward (an output wider than 64): sampled rows
    against the FP64 reference (BF16-representable inputs and weights)."""
    from paper_2411_05799_amd import native as N
    torch = _torch()
    rng = np.random.default_rng(12)
    B = 65536
    n_in, n_out = shape["n_in"], shape["n_out"]
    say(f"case: large batch forward {shape}")
    x = bf16_round(rng.normal(0.3, 1.7, size=(B, n_in))).astype(np.float32)
    s = N.Surrogate(max_batch=B, precision=N.SUR_BF16, training=False, seed=2, **shape)
    s.set_params(bf16_round(s.get_params()))
    ym, ys = rng.normal(size=n_out), rng.uniform(0.5, 2.0, size=n_out)
    s.set_norm(np.zeros(n_in), np.ones(n_in), ym, ys)
    p = s.get_params().astype(np.float64)
    out = torch.zeros((B, n_out), device="cuda")
    s.forward(_dev(x), out)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(B, 512, replace=False))
    f32 = np.float32
    shapes = M.layer_shapes(n_in, shape["n_hidden"], shape["n_hidden_layers"], n_out)
    ref = M.predict(p, shapes, x[rows].astype(np.float64), np.zeros(n_in), np.ones(n_in),
                    ym.astype(f32), ys.astype(f32))
    got = out.cpu().numpy()[rows].astype(np.float64)
    assert np.linalg.norm(got - ref) <= 1e-2 * np.linalg.norm(ref - ym.astype(f32))
    assert np.isfinite(out.cpu().numpy()).all()
    s.close()
