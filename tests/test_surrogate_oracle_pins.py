"""Pins of the surrogate's FP64 reference quantities (inputs, rollout update,
torque proxy) against closed forms and against the C oracle's own step."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import surrogate_oracle as S
from paper_2411_05799_amd import workloads as W

G = 9.81


def f32(v):
    """The float32 value the tables hold."""
    return float(np.float32(v))


def arm_robot(tip_z=0.5):
    """Torso: four 0.5 kg corner points on z = 0.  Arm: two points (0.4 kg at
    x = 0.3, 0.6 kg at x = 0.5) at height tip_z, hinged at (0.2, 0, tip_z) about +y."""
    pts = np.array([[-0.1, -0.1, 0, 0.5], [0.1, -0.1, 0, 0.5], [-0.1, 0.1, 0, 0.5],
                    [0.1, 0.1, 0, 0.5], [0.3, 0, tip_z, 0.4], [0.5, 0, tip_z, 0.6]], np.float32)
    joint = np.zeros((2, 8), np.float32)
    joint[1] = [0.2, 0, tip_z, 0, 1, 0, -W.NO_LIMIT, W.NO_LIMIT]
    return W.Morph(points=pts, pt_link=np.array([0, 0, 0, 0, 1, 1], np.int32),
                   parent=np.array([-1, 0], np.int32), joint=joint, name="arm")


def one_robot_workload(m, hf=None, ctrl=None):
    J = m.n_links - 1
    return W.Workload(params=W.Params(), hf=hf or W.flat_ground(), morphs=[m],
                      inst_morph=np.zeros(1, np.int32),
                      ctrl=[np.zeros((J, 3), np.float32) if ctrl is None else ctrl],
                      pose=np.array([[0, 0, 0, 1, 0, 0, 0]], np.float32), n_steps=1)


def row_at_rest(m, yaw=0.0, shift=(0.0, 0.0)):
    """State row with the torso frame at the origin (plus shift), turned by yaw."""
    y = m.points[:, :3].astype(np.float64)
    M = m.points[:, 3].astype(np.float64)
    gb = (M[:, None] * y).sum(0) / M.sum()
    Q = np.array([math.cos(yaw / 2), 0, 0, math.sin(yaw / 2)])
    c = S.quat_mat(Q) @ gb + [shift[0], shift[1], 0.0]
    row = np.zeros(13 + 2 * (m.n_links - 1))
    row[:3], row[3:7] = c, Q
    return row


def test_link_kinematics_match_the_c_oracle():
    m = W.hexapod()
    q = np.random.default_rng(0).uniform(-0.6, 0.6, m.n_links - 1)
    Rs, ts = S.link_transforms(m, q)
    y_ref, _, _, _ = O.OracleMorph(m).fk(q)
    y = np.array([Rs[l] @ p + ts[l] for p, l in zip(m.points[:, :3].astype(float), m.pt_link)])
    np.testing.assert_allclose(y, y_ref, atol=1e-14)


@pytest.mark.parametrize("yaw", [0.0, 1.1, -2.5])
def test_torque_of_a_horizontal_arm_is_its_weight_moment(yaw):
    m = arm_robot()
    so = S.SurrogateOracle(one_robot_workload(m))
    tau, _ = so.torque(0, row_at_rest(m, yaw))
    want = ((f32(0.3) - f32(0.2)) * f32(0.4) + (f32(0.5) - f32(0.2)) * f32(0.6)) * G
    assert abs(tau - want) < 1e-12


def test_torque_with_the_arm_resting_on_the_ground():
    """The tip points also carry a share M g / 6 of the weight."""
    m = arm_robot(tip_z=0.001)
    so = S.SurrogateOracle(one_robot_workload(m))
    tau, ambiguous = so.torque(0, row_at_rest(m, 0.3, shift=(0.7, -0.2)))
    f = (4 * 0.5 + f32(0.4) + f32(0.6)) * G / 6
    d1, d2 = f32(0.3) - f32(0.2), f32(0.5) - f32(0.2)
    assert not ambiguous
    assert abs(tau - abs(d1 * (f32(0.4) * G - f) + d2 * (f32(0.6) * G - f))) < 1e-12


def test_torque_sums_the_loads_of_distal_subtrees():
    # a chain torso -> a -> b along x: joint a carries both links' weight moments
    pts = np.array([[0, 0, 0, 1.0], [0.2, 0, 0.3, 0.5], [0.4, 0, 0.3, 0.25]], np.float32)
    joint = np.zeros((3, 8), np.float32)
    joint[1] = [0.1, 0, 0.3, 0, 1, 0, -W.NO_LIMIT, W.NO_LIMIT]
    joint[2] = [0.3, 0, 0.3, 0, 1, 0, -W.NO_LIMIT, W.NO_LIMIT]
    m = W.Morph(points=pts, pt_link=np.array([0, 1, 2], np.int32),
                parent=np.array([-1, 0, 1], np.int32), joint=joint)
    so = S.SurrogateOracle(one_robot_workload(m))
    tau, _ = so.torque(0, row_at_rest(m))
    a1, a2 = f32(0.1), f32(0.3)
    t1 = ((f32(0.2) - a1) * 0.5 + (f32(0.4) - a1) * 0.25) * G
    t2 = (f32(0.4) - a2) * 0.25 * G
    assert abs(tau - (t1 + t2) / 2) < 1e-12


def step_terrain():
    """Height 0 for x < 0 and 0.1 m for x >= 0 (cells of 2 cm from -1.28 m)."""
    nx = ny = 128
    H = np.zeros((ny, nx), np.float32)
    H[:, 64:] = 0.1
    return W.Heightfield(nx=nx, ny=ny, s=50.0, x0=-1.28, y0=-1.28, H=H)


def test_patch_follows_heading_on_a_step():
    m = arm_robot()
    so = S.SurrogateOracle(one_robot_workload(m, hf=step_terrain()))
    J = 1
    base = 13 + 12 * J
    row = row_at_rest(m)
    row[:2] = [0.01, 0.0]
    x = so.features(0, row, 0)
    patch = x[base:base + 64].reshape(8, 8)          # [a][b]
    want = np.zeros((8, 8))
    want[:4, :] = -0.1                                # behind the CoG: off the step
    np.testing.assert_allclose(patch, want, atol=1e-7)
    assert abs(x[2] - (row[2] - 0.1)) < 1e-7
    # turned a quarter to the left: "left" (b > 3.5) now points to -x
    row = row_at_rest(m, yaw=math.pi / 2)
    row[:2] = [0.01, 0.0]
    patch = so.features(0, row, 0)[base:base + 64].reshape(8, 8)
    want = np.zeros((8, 8))
    want[:, 4:] = -0.1
    np.testing.assert_allclose(patch, want, atol=1e-7)


def test_targets_and_rollout_update_match_the_oracle_step():
    """Commanded angles in the input are what the next ten oracle steps apply,
    and the update with the true delta reproduces the state ten steps on."""
    w = W.config1(seed=4)
    so = S.SurrogateOracle(w)
    ow = O.OracleWorld(w)
    st = ow.init_state(0)
    ow.run(0, st, 137)
    n = int(st[O.STEP])
    m = w.morphs[0]
    Jn = m.n_links - 1
    row0 = S.state_row(st, Jn, so.J)
    x = so.features(0, row0, n)
    np.testing.assert_allclose(x[13 + so.J:13 + 2 * so.J],
                               (row0[13:13 + so.J] - row0[13 + so.J:]) / w.params.dt)
    for k in range(S.HORIZON):
        ow.step(0, st)
        q = st[O.HDR:O.HDR + Jn]
        np.testing.assert_allclose(x[13 + 2 * so.J + k * so.J:13 + 2 * so.J + k * so.J + Jn], q,
                                   rtol=0, atol=1e-15)
    row10 = S.state_row(st, Jn, so.J)
    out = so.advance(0, row0, so.delta(row0, row10), n)
    np.testing.assert_allclose(out[:13], row10[:13], atol=1e-12)
    np.testing.assert_array_equal(out[13:], row10[13:])


def _yawed(row, yaw):
    """The same state turned by yaw about the world z axis through the origin."""
    Rz = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]])
    out = np.array(row, dtype=np.float64)
    for k in (0, 7, 10):
        out[k:k + 3] = Rz @ row[k:k + 3]
    out[3:7] = S.quat_mul([math.cos(yaw / 2), 0, 0, math.sin(yaw / 2)], row[3:7])
    return out


def test_heading_frame_inputs_do_not_depend_on_yaw():
    w = W.config1(seed=2)
    so = S.SurrogateOracle(w)
    ow = O.OracleWorld(w)
    st = ow.init_state(0)
    ow.run(0, st, 400)
    row = S.state_row(st, 18, so.J)
    base = so.features(0, row, 400)
    for yaw in (0.7, -2.9, 3.1):
        np.testing.assert_allclose(so.features(0, _yawed(row, yaw), 400), base, atol=1e-12)
    # a negated orientation quaternion is the same state
    neg = np.array(row)
    neg[3:7] *= -1
    np.testing.assert_allclose(so.features(0, neg, 400), base, atol=1e-15)


def test_heading_frame_closed_form_and_round_trip():
    hf = S.HeadingFrame([math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)])   # facing +y
    b = np.zeros(13)
    b[3], b[7:10], b[10:13] = 1.0, [0, 1.0, 0.25], [0.5, 0, 2.0]
    out = hf.to_frame(b)
    np.testing.assert_allclose(out[7:10], [1.0, 0, 0.25], atol=1e-15)      # moving forward
    np.testing.assert_allclose(out[10:13], [0, -0.5, 2.0], atol=1e-15)     # rolling to the right
    np.testing.assert_allclose(hf.from_frame(out), b, atol=1e-15)
    # the orientation itself becomes level and unturned, w >= 0
    Q = np.array([-math.cos(1.2), 0, 0, -math.sin(1.2)])
    h = S.HeadingFrame(Q)
    np.testing.assert_allclose(h.sign * S.quat_mul(h.q_minus, Q), [1, 0, 0, 0], atol=1e-15)
