"""GPU parity of the surrogate's simulator-side kernels (state rows, network
inputs, deltas, rollout update, torque proxy, native rollout) against the FP64
reference, through the C ABI."""
import numpy as np
import pytest

from oracle import surrogate_oracle as SO

pytestmark = pytest.mark.gpu

N_INST = 192


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def walked():
    """A world of hexapods on the octave terrain, 300 frames on."""
    import torch
    from paper_2411_05799_amd import native as N
    from paper_2411_05799_amd import workloads as W
    w = W.config2(n_inst=N_INST, n_steps=300)
    gw = N.World(w)
    gw.step_n(300)
    sw, fw = gw.sur_widths()
    rows = torch.zeros((N_INST, sw), device="cuda")
    gw.rows(rows)
    torch.cuda.synchronize()
    yield w, gw, rows
    gw.close()


def test_widths_and_rows_match_read_state(walked):
    from paper_2411_05799_amd import native as N
    w, gw, rows = walked
    assert gw.sur_widths() == (49, 293)
    r = rows.cpu().numpy()
    np.testing.assert_array_equal(r[:, :13], gw.read_state(N.F_BODY).T)
    np.testing.assert_array_equal(r[:, 13:31], gw.read_state(N.F_JOINT).T)
    np.testing.assert_array_equal(r[:, 31:], gw.read_state(N.F_JOINT_PREV).T)


def test_set_rows_inverts_rows(walked):
    import torch
    from paper_2411_05799_amd import native as N
    w, gw, rows = walked
    say("case: set_rows then rows on a fresh world, strided buffer")
    gw2 = N.World(w)
    buf = torch.full((N_INST, 64), 7.0, device="cuda")
    buf[:, :49] = rows
    gw2.set_rows(buf[:, :49])
    back = torch.zeros_like(rows)
    gw2.rows(back)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back.cpu().numpy(), rows.cpu().numpy())
    np.testing.assert_array_equal(gw2.read_state(N.F_BODY).T, rows[:, :13].cpu().numpy())
    assert np.all(gw2.read_state(N.F_STEP) == 0)
    gw2.close()


def test_features_match_reference(walked):
    import torch
    w, gw, rows = walked
    say("case: features, 192 hexapods at frame 300")
    x_world = torch.full((N_INST, 300), 9.0, device="cuda")
    x_rows = torch.full((N_INST, 300), 9.0, device="cuda")
    gw.sur_features(x_world[:, :293])
    gw.sur_features(x_rows[:, :293], s=rows, frame=300)
    torch.cuda.synchronize()
    a, b = x_world.cpu().numpy(), x_rows.cpu().numpy()
    np.testing.assert_array_equal(a, b)
    assert np.all(a[:, 293:] == 9.0)
    so = SO.SurrogateOracle(w)
    r = rows.cpu().numpy().astype(np.float64)
    J = 18
    checked = 0
    for i in range(N_INST):
        ref = so.features(i, r[i], 300)
        got = a[i, :293].astype(np.float64)
        np.testing.assert_allclose(got[:13][[0, 1]], 0.0)
        np.testing.assert_allclose(got[3:13], ref[3:13], rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(got[13:13 + J], ref[13:13 + J], rtol=0, atol=0)
        np.testing.assert_allclose(got[13 + J:13 + 2 * J], ref[13 + J:13 + 2 * J], atol=1e-4)
        np.testing.assert_allclose(got[13 + 2 * J:13 + 12 * J], ref[13 + 2 * J:13 + 12 * J],
                                   atol=2e-6)
        if so.near_edge(r[i, 0], r[i, 1]):
            continue
        assert abs(got[2] - ref[2]) <= 1e-6
        for k, (px, py) in enumerate(so.patch_points(r[i])):
            if so.near_edge(px, py):
                continue
            assert abs(got[13 + 12 * J + k] - ref[13 + 12 * J + k]) <= 1e-6, (i, k)
            checked += 1
    assert checked > 0.9 * N_INST * 64


def test_delta_and_advance(walked):
    import torch
    w, gw, rows = walked
    from paper_2411_05799_amd import native as N
    say("case: delta and rollout update over frames 300..309")
    gw2 = N.World(w)
    gw2.write_state(N.F_BODY, rows[:, :13].T.contiguous())
    gw2.write_state(N.F_JOINT, rows[:, 13:31].T.contiguous())
    gw2.write_state(N.F_JOINT_PREV, rows[:, 31:].T.contiguous())
    gw2.write_state(N.F_STEP, np.full(N_INST, 300, np.int32))
    gw2.step_n(10)
    y = torch.zeros((N_INST, 49), device="cuda")
    gw2.sur_delta(rows, y)
    after = torch.zeros_like(rows)
    gw2.rows(after)
    torch.cuda.synchronize()
    so = SO.SurrogateOracle(w)
    yd, ad, rd = y.cpu().numpy(), after.cpu().numpy(), rows.cpu().numpy()
    np.testing.assert_array_equal(yd[:, 13:], ad[:, 13:] - rd[:, 13:])
    for i in range(N_INST):   # body rows in the heading frame of the first state
        ref = so.delta(rd[i].astype(np.float64), ad[i].astype(np.float64))
        np.testing.assert_allclose(yd[i, :13], ref[:13], rtol=1e-5, atol=1e-6)
    # the update with the true delta lands on the stepped state; q, q_prev exactly
    s = rows.clone()
    gw2.sur_advance(s, y, 300)
    torch.cuda.synchronize()
    got, want = s.cpu().numpy(), after.cpu().numpy()
    np.testing.assert_array_equal(got[:, 13:], want[:, 13:])
    np.testing.assert_allclose(got[:, :13], want[:, :13], atol=2e-6)
    # and matches the FP64 update on the same inputs
    r, d = rows.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    for i in range(0, N_INST, 7):
        ref = so.advance(i, r[i], d[i], 300)
        np.testing.assert_allclose(got[i], ref, atol=2e-6)
    gw2.close()


def test_torque_matches_reference(walked):
    import torch
    w, gw, rows = walked
    say("case: torque proxy, 192 hexapods")
    acc_w = torch.zeros(N_INST, device="cuda")
    acc_r = torch.full((N_INST,), 1.0, device="cuda")
    gw.sur_torque(acc_w)
    gw.sur_torque(acc_r, s=rows, accumulate=True)
    torch.cuda.synchronize()
    a = acc_w.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(acc_r.cpu().numpy(), (acc_w + 1.0).cpu().numpy())
    so = SO.SurrogateOracle(w)
    r = rows.cpu().numpy().astype(np.float64)
    compared = 0
    for i in range(N_INST):
        tau, ambiguous = so.torque(i, r[i])
        if ambiguous:
            continue        # a load decision that float32 may take either way
        assert abs(a[i] - tau) <= 1e-4 * max(1.0, tau), (i, a[i], tau)
        compared += 1
    assert compared >= 0.8 * N_INST, compared
    assert np.all(a > 0) and np.all(np.isfinite(a))


def test_native_rollout_equals_composed_calls(walked):
    import torch
    from paper_2411_05799_amd import native as N
    w, gw, rows = walked
    say("case: native rollout vs composed calls, 3 calls")
    net = N.Surrogate(293, 256, 3, 49, max_batch=N_INST, training=False, seed=5)
    rng = np.random.default_rng(0)
    net.set_norm(rng.normal(0, 0.1, 293), rng.uniform(0.5, 2, 293), np.zeros(49),
                 np.full(49, 1e-3))
    s1, s2 = rows.clone(), rows.clone()
    x = torch.zeros((N_INST, 293), device="cuda")
    y = torch.zeros((N_INST, 49), device="cuda")
    t1 = torch.zeros(N_INST, device="cuda")
    t2 = torch.zeros(N_INST, device="cuda")
    gw.sur_rollout(net, s1, 300, 3, x, y, t1)
    for c in range(3):
        f = 300 + 10 * c
        gw.sur_features(x, s=s2, frame=f)
        net.forward(x, y)
        gw.sur_advance(s2, y, f)
        gw.sur_torque(t2, s=s2, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s1.cpu().numpy(), s2.cpu().numpy())
    np.testing.assert_array_equal(t1.cpu().numpy(), t2.cpu().numpy())
    assert not torch.equal(s1, rows)
    small = N.Surrogate(293, 64, 1, 49, max_batch=N_INST - 1, training=False)
    with pytest.raises(N.NpxError, match="batch limit"):
        gw.sur_rollout(small, s1, 300, 1, x, y)
    wrong = N.Surrogate(290, 64, 1, 49, max_batch=N_INST, training=False)
    with pytest.raises(N.NpxError, match="does not fit"):
        gw.sur_rollout(wrong, s1, 300, 1, x, y)
    net.close()
    small.close()
    wrong.close()


def test_advance_needs_joints_every_frame():
    import torch
    from paper_2411_05799_amd import native as N
    from paper_2411_05799_amd import workloads as W
    w = W.config2(n_inst=4, n_steps=10)
    w.params.K = 2
    gw = N.World(w)
    s = torch.zeros((4, 49), device="cuda")
    with pytest.raises(N.NpxError):
        gw.sur_advance(s, s, 0)
    gw.close()


def test_torque_uneven_robots_with_more_than_32_links():
    """Random legged robots, some with 33 links: the proxy runs one robot per
    64-lane wave (at most 32 links: two per wave); against the reference."""
    import torch
    from paper_2411_05799_amd import native as N
    from paper_2411_05799_amd import workloads as W
    w = W.config3(n_inst=96, n_steps=200)
    l_max = max(m.n_links for m in w.morphs)
    assert l_max > 32, l_max
    say(f"case: torque proxy, 96 uneven robots, up to {l_max} links")
    gw = N.World(w)
    gw.step_n(200)
    sw, _ = gw.sur_widths()
    rows = torch.zeros((96, sw), device="cuda")
    gw.rows(rows)
    acc = torch.zeros(96, device="cuda")
    gw.sur_torque(acc, s=rows)
    torch.cuda.synchronize()
    flags = gw.read_state(N.F_FLAGS)
    gw.close()
    a = acc.cpu().numpy().astype(np.float64)
    so = SO.SurrogateOracle(w)
    r = rows.cpu().numpy().astype(np.float64)
    compared = 0
    for i in range(96):
        if flags[i] != 0:
            continue
        tau, ambiguous = so.torque(i, r[i])
        if ambiguous:
            continue
        assert abs(a[i] - tau) <= 1e-4 * max(1.0, tau), (i, a[i], tau)
        compared += 1
    assert compared >= 0.6 * 96, compared


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_native_rollout_fused_network_and_fp32(precision):
    """256 robots (whole 128-row blocks): the BF16 network runs as one fused
    kernel inside the rollout and inside npx_sur_forward alike, the FP32 one
    layer by layer with float inputs; the native rollout equals the composed
    calls bit for bit in both."""
    import torch
    from paper_2411_05799_amd import native as N
    from paper_2411_05799_amd import workloads as W
    say(f"case: native rollout vs composed calls, 256 robots, {precision}")
    I = 256
    w = W.config2(n_inst=I, n_steps=100)
    gw = N.World(w)
    gw.step_n(100)
    sw, fw = gw.sur_widths()
    rows = torch.zeros((I, sw), device="cuda")
    gw.rows(rows)
    prec = N.SUR_BF16 if precision == "bf16" else N.SUR_FP32
    net = N.Surrogate(fw, 384, 2, sw, max_batch=I, precision=prec, training=False, seed=7)
    rng = np.random.default_rng(1)
    net.set_norm(rng.normal(0, 0.1, fw), rng.uniform(0.5, 2, fw), np.zeros(sw),
                 np.full(sw, 1e-3))
    s1, s2 = rows.clone(), rows.clone()
    x = torch.zeros((I, fw), device="cuda")
    y = torch.zeros((I, sw), device="cuda")
    t1 = torch.zeros(I, device="cuda")
    t2 = torch.zeros(I, device="cuda")
    gw.sur_rollout(net, s1, 100, 4, x, y, t1)
    for c in range(4):
        f = 100 + 10 * c
        gw.sur_features(x, s=s2, frame=f)
        net.forward(x, y)
        gw.sur_advance(s2, y, f)
        gw.sur_torque(t2, s=s2, accumulate=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(s1.cpu().numpy(), s2.cpu().numpy())
    np.testing.assert_array_equal(t1.cpu().numpy(), t2.cpu().numpy())
    assert not torch.equal(s1, rows) and torch.isfinite(s1).all()
    net.close()
    gw.close()
