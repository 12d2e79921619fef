"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the step to something other than the oracle
itself: a closed form, an invariant, a textbook routine (numpy lstsq, SVD) or
brute force on tiny inputs. They are chosen so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails at least one.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_05799_amd import workloads as W

G0 = 9.81
HALF_Z = float(np.float32(0.05 / 2))   # bottom corners of the default box sit at -HALF_Z


# ----------------------------------------------------------------------------
# helpers: tiny scenes written as workload tables
# ----------------------------------------------------------------------------

def box_morph(lx=0.2, ly=0.1, lz=0.05, mass=1.0):
    """A box as the paper's createBox makes it: its 8 corner points (Sec. IV-A)."""
    pts = np.array([[sx * lx / 2, sy * ly / 2, sz * lz / 2, mass / 8]
                    for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], dtype=np.float32)
    return W.Morph(points=pts, pt_link=np.zeros(8, np.int32), parent=np.array([-1], np.int32),
                   joint=np.zeros((1, 8), np.float32), name="box8")


def scene(morph, pose, params=None, hf=None, ctrl=None):
    w = W.Workload(params=params or W.Params(), hf=hf or W.flat_ground(), morphs=[morph],
                   inst_morph=np.zeros(1, np.int32),
                   ctrl=[ctrl if ctrl is not None else np.zeros((morph.n_joints, 3), np.float32)],
                   pose=np.asarray(pose, np.float32)[None, :])
    return O.OracleWorld(w)


def energy(ow, st, params):
    """E = kinetic + rotational + gravity potential + penalty spring energy."""
    m = ow.morph_of(0)
    J = m.n_joints
    _, gb, Ib, M = m.fk(st[O.HDR:O.HDR + J])
    Q = st[O.Q_:O.Q_ + 4]
    R = quat_mat(Q)
    Iw = R @ Ib @ R.T
    v, w = st[O.V_:O.V_ + 3], st[O.W_:O.W_ + 3]
    c = st[O.C_:O.C_ + 3]
    P = ow.points(0, st)
    spring = 0.0
    for p in P:
        d = ow.params.height(p[0], p[1]) - p[2]
        if d > 0:
            spring += 0.5 * params.k_n * d * d
    g = np.asarray(params.g)
    return 0.5 * M * v @ v + 0.5 * w @ Iw @ w - M * g @ c + spring


def quat_mat(Q):
    w, x, y, z = Q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def kabsch(A, B):
    """Rotation R and translation t minimising |R A + t - B| (SVD; textbook)."""
    ca, cb = A.mean(0), B.mean(0)
    H = (A - ca).T @ (B - cb)
    U, _, Vt = np.linalg.svd(H)
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, cb - R @ ca


# ----------------------------------------------------------------------------
# S1: height-map look-up vs brute force
# ----------------------------------------------------------------------------

def test_cell_lookup_brute_force():
    rng = np.random.default_rng(11)
    nx, ny, s, x0, y0 = 5, 4, 10.0, -0.23, 0.4
    H = rng.normal(size=(ny, nx)).astype(np.float32)
    hf = W.Heightfield(nx=nx, ny=ny, s=s, x0=x0, y0=y0, H=H)
    P = O.OracleParams(W.Params(), hf)

    def brute(u0, cell, n, x):
        # linear scan over the cell intervals [u0 + i/s, u0 + (i+1)/s); outside -> edge cell
        if x < u0 + cell:
            return 0
        for i in range(n):
            if u0 + i * cell <= x < u0 + (i + 1) * cell:
                return i
        return n - 1

    checked = 0
    for _ in range(2000):
        x = rng.uniform(x0 - 0.3, x0 + nx / s + 0.3)
        y = rng.uniform(y0 - 0.3, y0 + ny / s + 0.3)
        # skip points within double rounding of an edge
        ex = abs(s * (x - x0) - round(s * (x - x0)))
        ey = abs(s * (y - y0) - round(s * (y - y0)))
        if ex < 1e-9 or ey < 1e-9:
            continue
        i, j = P.cell(x, y)
        assert (i, j) == (brute(x0, 1 / s, nx, x), brute(y0, 1 / s, ny, y))
        assert P.height(x, y) == float(H[j, i])
        checked += 1
    assert checked > 1900
    # flat plane: one cell, every look-up is 0 (d = -z)
    Pf = O.OracleParams(W.Params(), W.flat_ground())
    assert Pf.height(123.4, -99.0) == 0.0 and Pf.cell(1e9, -1e9) == (0, 0)
    assert Pf.cell(float("nan"), 0.0) == (0, 0)


# ----------------------------------------------------------------------------
# S6: the friction least squares
# ----------------------------------------------------------------------------

def lstsq_ref(src, dst):
    n = len(src)
    A = np.zeros((2 * n, 3))
    b = np.zeros(2 * n)
    A[0::2, 0] = 1.0
    A[0::2, 2] = -src[:, 1]
    A[1::2, 1] = 1.0
    A[1::2, 2] = src[:, 0]
    b[0::2] = dst[:, 0] - src[:, 0]
    b[1::2] = dst[:, 1] - src[:, 1]
    return np.linalg.lstsq(A, b, rcond=None)[0]


@pytest.mark.parametrize("n", [2, 3, 7, 40])
def test_lsq_equals_lstsq(n):
    rng = np.random.default_rng(n)
    src = rng.normal(scale=0.2, size=(n, 2))
    dst = src + rng.normal(scale=0.01, size=(n, 2))
    a, k = O.lsq(src, dst)
    assert k == 3
    np.testing.assert_allclose(a, lstsq_ref(src, dst), rtol=0, atol=1e-12)


def test_lsq_rigid_closed_form():
    rng = np.random.default_rng(5)
    src = rng.normal(scale=0.3, size=(12, 2))
    for alpha in (0.3, -0.05, 1e-4):
        t = np.array([0.02, -0.01])
        R = np.array([[math.cos(alpha), -math.sin(alpha)], [math.sin(alpha), math.cos(alpha)]])
        dst = src @ R.T + t
        a, _ = O.lsq(src, dst)
        assert abs(a[2] - math.sin(alpha)) < 1e-12
        np.testing.assert_allclose(a[:2], t + (math.cos(alpha) - 1) * src.mean(0), atol=1e-12)


def test_lsq_translation_covariance_and_degenerate():
    rng = np.random.default_rng(6)
    src = rng.normal(scale=0.3, size=(9, 2))
    t = np.array([1e-3, 2e-3])
    a, _ = O.lsq(src, src + t)
    np.testing.assert_allclose(a, [t[0], t[1], 0.0], atol=1e-13)
    # origin covariance: shift both sets by o -> a3 unchanged, a -> a - a3 J o
    dst = src + rng.normal(scale=0.01, size=src.shape)
    o = np.array([0.7, -1.3])
    a0, _ = O.lsq(src, dst)
    a1, _ = O.lsq(src + o, dst + o)
    Jo = np.array([-o[1], o[0]])
    assert abs(a1[2] - a0[2]) < 1e-12
    np.testing.assert_allclose(a1[:2], a0[:2] - a0[2] * Jo, atol=1e-12)
    # one pair: translation only
    a, k = O.lsq(src[:1], dst[:1])
    assert k == 2 and a[2] == 0.0
    np.testing.assert_allclose(a[:2], dst[0] - src[0], atol=1e-15)
    # no spread (coincident points): translation only
    a, k = O.lsq(np.repeat(src[:1], 5, 0), np.repeat(dst[:1], 5, 0))
    assert k == 2 and a[2] == 0.0
    # empty set
    a, k = O.lsq(np.zeros((0, 2)), np.zeros((0, 2)))
    assert k == 0 and not a.any()


# ----------------------------------------------------------------------------
# FK / joint-angle determination and mass properties
# ----------------------------------------------------------------------------

def test_fk_zero_pose_and_joint_recovery():
    m = W.hexapod()
    om = O.OracleMorph(m)
    y0, g0, I0, M = om.fk(np.zeros(18))
    np.testing.assert_array_equal(y0, m.points[:, :3].astype(np.float64))
    assert abs(M - 4.1) < 1e-6
    rng = np.random.default_rng(3)
    q = rng.uniform(-0.6, 0.6, size=18)
    y, gb, Ib, _ = om.fk(q)
    rho = m.points[:, :3].astype(np.float64)
    # rigid transform of every link from its points (Kabsch), independent of the chain
    T = []
    for l in range(m.n_links):
        sel = m.pt_link == l
        T.append(kabsch(rho[sel], y[sel]))
    for l in range(1, m.n_links):
        p = m.parent[l]
        Rp, tp = T[p]
        Rl, tl = T[l]
        rel = Rp.T @ Rl                      # rotation of link l relative to its parent
        a = m.joint[l, 3:6].astype(np.float64)
        a /= np.linalg.norm(a)
        # the relative rotation is about the hinge axis ...
        np.testing.assert_allclose(rel @ a, a, atol=1e-12)
        # ... by the applied angle (signed, right-hand rule)
        e = np.cross(a, [1.0, 0.3, 0.1])
        e /= np.linalg.norm(e)
        ang = math.atan2(np.dot(a, np.cross(e, rel @ e)), np.dot(e, rel @ e))
        assert abs(ang - q[l - 1]) < 1e-10
        # the anchor stays attached to the parent
        o = m.joint[l, :3].astype(np.float64)
        np.testing.assert_allclose(Rl @ o + tl, Rp @ o + tp, atol=1e-12)
    # mass properties: per-link parallel-axis sum equals the point sum
    I_sum = np.zeros((3, 3))
    for l in range(m.n_links):
        sel = m.pt_link == l
        ml = m.points[sel, 3].astype(np.float64)
        cl = (ml[:, None] * rho[sel]).sum(0) / ml.sum()
        d = rho[sel] - cl
        Il = (ml[:, None, None] * ((d * d).sum(1)[:, None, None] * np.eye(3)
                                   - d[:, :, None] * d[:, None, :])).sum(0)
        Rl, tl = T[l]
        p = Rl @ cl + tl - gb
        I_sum += Rl @ Il @ Rl.T + ml.sum() * (p @ p * np.eye(3) - np.outer(p, p))
    np.testing.assert_allclose(Ib, I_sum, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(gb, (m.points[:, 3:4] * y).sum(0) / m.points[:, 3].sum(), atol=1e-14)


# ----------------------------------------------------------------------------
# S4: integration closed forms
# ----------------------------------------------------------------------------

def test_free_fall_discrete_parabola():
    z0, v0, n = 1000.0, 20.0, 5000   # |v| stays below the 50 m/s health bound
    ow = scene(box_morph(), [0.0, 0.0, z0, 1, 0, 0, 0])
    st = ow.init_state(0)
    st[O.V_ + 2] = v0
    c0 = st[O.C_:O.C_ + 3].copy()
    ow.run(0, st, n)
    dt = 1e-3
    z = c0[2] + n * dt * v0 - G0 * dt * dt * n * (n + 1) / 2
    assert abs(st[O.C_ + 2] - z) <= 1e-11 * abs(z)
    assert abs(st[O.V_ + 2] - (v0 - n * dt * G0)) < 1e-9
    # and within g dt t / 2 of the continuous parabola
    t = n * dt
    assert abs(st[O.C_ + 2] - (c0[2] + v0 * t - 0.5 * G0 * t * t)) <= 0.5 * G0 * dt * t + 1e-9


def test_cog_invariance_under_joint_motion():
    """Joint updates never move the world CoG: a hexapod swinging its legs in free
    flight follows the passive body's parabola bit for bit, and its joints read the
    commanded sinusoid."""
    w1 = W.config1(seed=7)
    pose = np.array([0.0, 0.0, 50.0, 1, 0, 0, 0], np.float32)
    active = O.OracleWorld(W.Workload(params=w1.params, hf=w1.hf, morphs=w1.morphs,
                                      inst_morph=w1.inst_morph, ctrl=w1.ctrl, pose=pose[None]))
    passive = scene(box_morph(), pose)
    sa, sp = active.init_state(0), passive.init_state(0)
    sp[O.C_:O.C_ + 3] = sa[O.C_:O.C_ + 3]
    for n in range(2000):
        active.step(0, sa)
        passive.step(0, sp)
        assert np.array_equal(sa[O.C_:O.C_ + 3], sp[O.C_:O.C_ + 3])
    np.testing.assert_array_equal(sa[O.Q_:O.Q_ + 4], [1, 0, 0, 0])
    ctrl = w1.ctrl[0].astype(np.float64)
    t = 1999 * 1e-3
    qh = ctrl[:, 0] * np.sin(2 * np.pi * ctrl[:, 1] * t + ctrl[:, 2])
    np.testing.assert_allclose(sa[O.HDR:O.HDR + 18], qh, atol=1e-14)


def test_yaw_integration_exact_exponential():
    ow = scene(box_morph(), [0.0, 0.0, 100.0, 1, 0, 0, 0])
    st = ow.init_state(0)
    st[O.W_ + 2] = 1.0   # spin about a principal axis: no gyroscopic torque
    n = 3000
    ow.run(0, st, n)
    a = n * 1e-3 * 1.0
    np.testing.assert_allclose(st[O.Q_:O.Q_ + 4], [math.cos(a / 2), 0, 0, math.sin(a / 2)],
                               atol=1e-12)
    np.testing.assert_allclose(st[O.W_:O.W_ + 3], [0, 0, 1.0], atol=1e-12)


def test_torque_free_rotation_conserves_momentum():
    """Euler's equations without torque: world angular momentum is conserved; the
    explicit gyroscopic term keeps the drift first order in dt."""
    m = box_morph(0.3, 0.2, 0.05, 2.0)
    drift = []
    for dt in (1e-3, 5e-4):
        ow = scene(m, [0.0, 0.0, 100.0, 1, 0, 0, 0], params=W.Params(dt=dt))
        st = ow.init_state(0)
        st[O.W_:O.W_ + 3] = [3.0, 0.5, 4.0]

        def L(s):
            _, _, Ib, _ = ow.morph_of(0).fk(np.zeros(0))
            R = quat_mat(s[O.Q_:O.Q_ + 4])
            return R @ Ib @ R.T @ s[O.W_:O.W_ + 3]

        L0 = L(st)
        ow.run(0, st, int(round(0.5 / dt)))
        drift.append(np.linalg.norm(L(st) - L0) / np.linalg.norm(L0))
    assert drift[0] < 2e-2
    assert 1.6 < drift[0] / drift[1] < 2.4   # first order in dt


# ----------------------------------------------------------------------------
# S2 + contact: rest, drop, tilt recovery
# ----------------------------------------------------------------------------

def test_rest_is_an_equilibrium():
    p = W.Params()
    mass = 1.5
    d_eq = mass * G0 / (4 * p.k_n)
    ow = scene(box_morph(mass=mass), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_ + 2] = HALF_Z - d_eq
    E0 = energy(ow, st, p)
    c0 = st[:13].copy()
    for _ in range(10):
        ow.run(0, st, 1000)
        assert abs(energy(ow, st, p) - E0) <= 1e-12 * abs(E0)
    np.testing.assert_allclose(st[:13], c0, atol=1e-12)


def test_drop_has_no_energy_gain_and_settles():
    p = W.Params()
    h0 = 0.05
    d_eq = 1.0 * G0 / (4 * p.k_n)
    ow = scene(box_morph(), [0.0, 0.0, HALF_Z + h0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    E0 = energy(ow, st, p)
    Emax = E0
    for _ in range(3000):
        ow.step(0, st)
        Emax = max(Emax, energy(ow, st, p))
    assert Emax <= E0 + 1e-3 * 1.0 * G0 * h0
    assert abs(st[O.C_ + 2] - (HALF_Z - d_eq)) < 1e-6
    assert np.linalg.norm(st[O.V_:O.V_ + 3]) < 1e-6


def test_tilted_box_lands_level():
    """Normal-force torques turn a tilted box flat (a wrong torque sign tips it over)."""
    p = W.Params()
    a = 0.2
    pose = [0.0, 0.0, 0.08, math.cos(a / 2), math.sin(a / 2), 0.0, 0.0]
    ow = scene(box_morph(), pose, params=p)
    st = ow.init_state(0)
    ow.run(0, st, 4000)
    Q = st[O.Q_:O.Q_ + 4]
    tilt = 2 * math.acos(min(1.0, math.sqrt(Q[0] ** 2 + Q[3] ** 2)))
    assert tilt < 1e-4
    assert st[O.FLAGS] == 0
    d = ow.step(0, st, diag=True)
    assert d[O.D_NC] == 4


# ----------------------------------------------------------------------------
# S5-S8: static friction -- incline stick/slide, spin stop
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("mu", [0.3, 0.5, 1.0])
@pytest.mark.parametrize("side", [-1, +1])
def test_incline_stick_slide_threshold(mu, side):
    """A block on a plane under gravity tilted by theta sticks iff tan(theta) <= mu;
    beyond it slides with x_n = g (sin - mu cos) dt^2 n (n+1) / 2 (Coulomb)."""
    theta = math.atan(mu) * (1 + side * 1e-3)
    g = (G0 * math.sin(theta), 0.0, -G0 * math.cos(theta))
    p = W.Params(g=g, mu=mu)
    mass = 1.0
    d_eq = mass * G0 * math.cos(theta) / (4 * p.k_n)
    ow = scene(box_morph(mass=mass), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
    n = 10_000
    x0 = st[O.C_]
    ow.run(0, st, n)
    dx = st[O.C_] - x0
    if side < 0:
        assert abs(dx) < 1e-11
        assert abs(st[O.V_]) < 1e-12
    else:
        dt = p.dt
        xn = G0 * (math.sin(theta) - mu * math.cos(theta)) * dt * dt * n * (n + 1) / 2
        assert xn > 0
        assert abs(dx - xn) <= 1e-9 * xn + 1e-13
    assert abs(st[O.C_ + 1]) < 1e-12          # no sideways drift
    np.testing.assert_allclose(st[O.Q_:O.Q_ + 4], [1, 0, 0, 0], atol=1e-12)


def test_stick_step_leaves_no_velocity():
    theta = 0.2
    p = W.Params(g=(G0 * math.sin(theta), 0.0, -G0 * math.cos(theta)), mu=1.0)
    d_eq = G0 * math.cos(theta) / (4 * p.k_n)
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
    d = ow.step(0, st, diag=True)
    assert d[O.D_LAMBDA] == 1.0 and d[O.D_NS] == 4
    assert abs(d[O.D_FF] - G0 * math.sin(theta)) < 1e-9   # estimated friction = M g sin
    # the trial velocity dt g sin(theta) ~ 2e-3 m/s is removed to rounding of point
    # coordinates (~1e-17 m) over dt
    assert np.abs(st[O.V_:O.V_ + 2]).max() < 1e-13
    assert abs(st[O.V_ + 2]) < 1e-14


def test_infinite_mu_never_slides():
    theta = 1.2   # tan = 2.6
    p = W.Params(g=(G0 * math.sin(theta), 0.0, -G0 * math.cos(theta)), mu=math.inf)
    d_eq = G0 * math.cos(theta) / (4 * p.k_n)
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
    ow.run(0, st, 5000)
    assert abs(st[O.C_]) < 1e-11


def test_spinning_box_stops_under_stick():
    """A box turning about z on the ground: contact points move rigidly, the fit
    recovers a3 = sin(dt w) and the correction removes the whole turn."""
    p = W.Params(mu=1.0)
    d_eq = G0 / (4 * p.k_n)
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
    st[O.W_ + 2] = 2.0
    d = ow.step(0, st, diag=True)
    assert d[O.D_NS] == 4 and d[O.D_LAMBDA] == 1.0
    assert abs(d[O.D_A + 2] - math.sin(2.0e-3)) < 1e-12
    assert abs(st[O.W_ + 2]) < 1e-9
    np.testing.assert_allclose(st[O.Q_:O.Q_ + 4], [1, 0, 0, 0], atol=1e-12)


def test_leaving_contact_has_no_friction():
    """Points touching now but not at t+1 are not in the friction set."""
    p = W.Params(mu=1.0)
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - 1e-4]
    st[O.V_:O.V_ + 3] = [0.5, 0.0, 1.0]
    d = ow.step(0, st, diag=True)
    assert d[O.D_NC] == 4 and d[O.D_NS] == 0 and d[O.D_LAMBDA] == 0.0
    assert st[O.V_] == 0.5


def test_health_flag_freezes_instance():
    ow = scene(box_morph(), [0.0, 0.0, 1.0, 1, 0, 0, 0])
    st = ow.init_state(0)
    st[O.V_] = 80.0
    ow.step(0, st)
    assert st[O.FLAGS] != 0
    frozen = st.copy()
    ow.run(0, st, 10)
    np.testing.assert_array_equal(st, frozen)
    st2 = ow.init_state(0)
    st2[O.W_] = float("nan")
    ow.step(0, st2)
    assert int(st2[O.FLAGS]) & 1


# ----------------------------------------------------------------------------
# workloads: seeded, deterministic inputs of the stated shapes
# ----------------------------------------------------------------------------

def test_workload_shapes_and_determinism():
    m = W.hexapod()
    assert m.n_points == 352 and m.n_links == 19
    assert abs(float(m.points[:, 3].astype(np.float64).sum()) - 4.1) < 1e-5
    w1, w2 = W.hexapod_batch(8, seed=2), W.hexapod_batch(8, seed=2)
    for a, b in zip(w1.ctrl, w2.ctrl):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(w1.hf.H, w2.hf.H)
    assert w1.hf.H.shape == (512, 512)
    assert float(np.abs(w1.hf.H).max()) <= 0.03 + 1e-6
    for i in range(4):
        r = np.random.default_rng(i)
        mm = W.random_legged(r)
        assert 200 <= mm.n_points <= 600
        assert mm.n_joints in (8, 12, 16, 18, 24, 32, 6 * 2, 6 * 4, 8 * 3, 4 * 3, 4 * 4, 8 * 2)
        assert np.all(np.bincount(mm.pt_link)[1:] >= 8)


def test_contact_is_strictly_below_the_table():
    """kappa = [h - z > 0]: a point exactly on the surface or above it is free."""
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0])
    for z_bottom, n_expect in ((0.0, 0), (5e-4, 0), (-1e-9, 4)):
        st = ow.init_state(0)
        st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z + z_bottom]
        d = ow.step(0, st, diag=True)
        assert d[O.D_NC] == n_expect, z_bottom


def test_friction_set_needs_contact_at_both_times():
    """A box rolling onto its other edge: two corners touch now, the other two only
    at the predicted t+1; only the first two enter the fit (eq. 3: points existing
    in both time steps)."""
    a = 0.01
    p = W.Params()
    ow = scene(box_morph(), [0.0, 0.0, 0.0, math.cos(a / 2), math.sin(a / 2), 0.0, 0.0], params=p)
    st = ow.init_state(0)
    P = ow.points(0, st)
    low = P[:, 2].min()
    st[O.C_ + 2] += -low - 1e-5          # lowest edge 10 um into the ground
    st[O.W_] = -10.0                      # turns the high edge down by 0.5 mm ...
    st[O.V_:O.V_ + 3] = [0.05, 0.0, -0.8]  # ... and sinks 0.8 mm: it touches at t+1 only
    P = ow.points(0, st)
    now = int((P[:, 2] < 0).sum())
    d = ow.step(0, st, diag=True)
    Ps = ow.points(0, st)
    assert now == 2 and d[O.D_NC] == 2
    assert d[O.D_NS] == 2
    assert (Ps[:, 2] < 0).sum() == 4      # all four bottom corners touch after the step


# ----------------------------------------------------------------------------
# force-weighted friction fit (closing remark of Sec. III-C)
# ----------------------------------------------------------------------------

def weighted_lstsq_ref(src, dst, w):
    """Each pair's two residual rows scaled by sqrt(w): the weighted least squares."""
    n = len(src)
    A = np.zeros((2 * n, 3))
    b = np.zeros(2 * n)
    A[0::2, 0] = 1.0
    A[0::2, 2] = -src[:, 1]
    A[1::2, 1] = 1.0
    A[1::2, 2] = src[:, 0]
    b[0::2] = dst[:, 0] - src[:, 0]
    b[1::2] = dst[:, 1] - src[:, 1]
    s = np.sqrt(np.repeat(w, 2))
    return np.linalg.lstsq(A * s[:, None], b * s, rcond=None)[0]


@pytest.mark.parametrize("n", [2, 3, 7, 40])
def test_weighted_lsq_equals_weighted_lstsq(n):
    rng = np.random.default_rng(100 + n)
    src = rng.normal(scale=0.2, size=(n, 2))
    dst = src + rng.normal(scale=0.01, size=(n, 2))
    w = rng.uniform(0.1, 5.0, size=n)
    a, k = O.lsq(src, dst, weights=w)
    assert k == 3
    np.testing.assert_allclose(a, weighted_lstsq_ref(src, dst, w), rtol=0, atol=1e-12)


def test_weighted_lsq_special_cases():
    rng = np.random.default_rng(7)
    src = rng.normal(scale=0.3, size=(8, 2))
    dst = src + rng.normal(scale=0.01, size=src.shape)
    # equal weights: the unweighted fit, whatever their size
    a0, _ = O.lsq(src, dst)
    a1, _ = O.lsq(src, dst, weights=np.full(8, 3.7))
    np.testing.assert_allclose(a1, a0, atol=1e-13)
    # a zero weight drops its pair
    w = rng.uniform(0.5, 2.0, size=8)
    w[3] = 0.0
    keep = np.arange(8) != 3
    a2, _ = O.lsq(src, dst, weights=w)
    a3, _ = O.lsq(src[keep], dst[keep], weights=w[keep])
    np.testing.assert_allclose(a2, a3, atol=1e-13)
    # data that the linear model fits exactly is fitted exactly for any weights
    t = np.array([0.01, -0.02])
    s3 = 0.05
    exact = src + np.stack([-s3 * src[:, 1], s3 * src[:, 0]], 1) + t
    a4, k = O.lsq(src, exact, weights=rng.uniform(0.1, 9.0, size=8))
    assert k == 3
    np.testing.assert_allclose(a4, [t[0], t[1], s3], atol=1e-13)
    # one weighted pair among zeros: no spread, its own slip
    w1 = np.zeros(8)
    w1[5] = 2.0
    a5, k = O.lsq(src, dst, weights=w1)
    assert k == 2 and a5[2] == 0.0
    np.testing.assert_allclose(a5[:2], dst[5] - src[5], atol=1e-15)
    # all weights zero: no motion
    a6, k = O.lsq(src, dst, weights=np.zeros(8))
    assert k == 0 and not a6.any()


def test_force_weighting_in_the_step():
    """Slips that come from one rigid trial motion (a box spinning and
    sliding, even tilted so that its corners press unequally) are fitted
    exactly by either sum, so the weighted step equals the unweighted one;
    joint motion makes the slips non-rigid and the weighting changes the
    fit (a hexapod walking on flat ground)."""
    for tilt in (0.0, 0.02):
        out = []
        for weighted in (False, True):
            p = W.Params(mu=1.0, friction_weighting=weighted)
            d_eq = G0 / (4 * p.k_n)
            q = [math.cos(tilt / 2), math.sin(tilt / 2), 0.0, 0.0]
            ow = scene(box_morph(), [0.0, 0.0, 0.0] + q, params=p)
            st = ow.init_state(0)
            st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
            st[O.W_ + 2] = 2.0
            st[O.V_] = 0.05
            d = ow.step(0, st, diag=True)
            out.append((d[O.D_A:O.D_A + 3].copy(), d[O.D_NS]))
        (a_u, n_u), (a_w, n_w) = out
        assert n_u == n_w >= 2
        np.testing.assert_allclose(a_w, a_u, rtol=0, atol=1e-14)
    ends = []
    for weighted in (False, True):
        w = W.config1(n_steps=400)
        w.params.friction_weighting = weighted
        ow = O.OracleWorld(w)
        st = ow.init_state(0)
        ow.run(0, st, 400)
        assert st[O.FLAGS] == 0 and np.isfinite(st[:13]).all()
        ends.append(st[:13].copy())
    assert np.abs(ends[1][:2] - ends[0][:2]).max() > 1e-6


# ----------------------------------------------------------------------------
# bilinear height-map option (a smoother ground than the look-up table)
# ----------------------------------------------------------------------------

def _table(H, s=50.0, x0=-1.0, y0=-2.0):
    ny, nx = H.shape
    return W.Heightfield(nx=nx, ny=ny, s=s, x0=x0, y0=y0, H=H.astype(np.float32))


def test_bilinear_reproduces_planes_and_centres():
    """Entries sampled from a plane at the cell centres give that plane exactly
    everywhere between the outer centres; at a centre the entry itself; the
    table look-up of the same map differs inside a cell."""
    nx, ny, s, x0, y0 = 7, 5, 50.0, -1.0, -2.0
    xc = x0 + (np.arange(nx) + 0.5) / s
    yc = y0 + (np.arange(ny) + 0.5) / s
    H = (0.25 * xc[None, :] - 0.5 * yc[:, None] + 0.125).astype(np.float32)
    hf = _table(H, s, x0, y0)
    bil = O.OracleParams(W.Params(hf_bilinear=True), hf)
    tab = O.OracleParams(W.Params(), hf)
    rng = np.random.default_rng(3)
    for x, y in zip(rng.uniform(xc[0], xc[-1], 50), rng.uniform(yc[0], yc[-1], 50)):
        # the plane through the stored (float32) entries
        i = min(int((x - x0) * s - 0.5), nx - 2)
        j = min(int((y - y0) * s - 0.5), ny - 2)
        fu, fw = (x - x0) * s - 0.5 - i, (y - y0) * s - 0.5 - j
        h = ((1 - fu) * (1 - fw) * H[j, i] + fu * (1 - fw) * H[j, i + 1] +
             (1 - fu) * fw * H[j + 1, i] + fu * fw * H[j + 1, i + 1])
        assert abs(bil.height(x, y) - h) < 1e-15
        assert abs(bil.height(x, y) - (0.25 * x - 0.5 * y + 0.125)) < 1e-7
    for i in range(nx):
        for j in range(ny):
            assert abs(bil.height(xc[i], yc[j]) - float(H[j, i])) < 1e-12
    assert abs(bil.height(xc[2] + 0.3 / s, yc[1]) - tab.height(xc[2] + 0.3 / s, yc[1])) > 1e-4


def test_bilinear_is_continuous_and_held_outside():
    rng = np.random.default_rng(4)
    H = rng.uniform(-0.03, 0.03, size=(6, 9)).astype(np.float32)
    hf = _table(H)
    bil = O.OracleParams(W.Params(hf_bilinear=True), hf)
    # across a cell edge (a table discontinuity) and across a centre line
    for x in (-1.0 + 3.0 / 50, -1.0 + 4.5 / 50):
        lo, hi = bil.height(x - 1e-12, -2.0 + 2.2 / 50), bil.height(x + 1e-12, -2.0 + 2.2 / 50)
        assert abs(lo - hi) < 1e-9
    # beyond the outer centres the height is held
    assert abs(bil.height(-5.0, -2.0 + 0.5 / 50) - float(H[0, 0])) < 1e-12
    assert bil.height(5.0, 5.0) == float(H[-1, -1])
    # a one-cell map (flat ground) reads its entry everywhere
    flat = O.OracleParams(W.Params(hf_bilinear=True), W.flat_ground())
    assert flat.height(0.3, -7.0) == 0.0


def test_bilinear_box_rests_on_a_slope_it_would_step_on():
    """A box on a table sampled from a gentle slope: with the bilinear reading
    the ground under the corners is the plane, so the box settles without
    falling off cell steps; rest heights follow the plane."""
    nx = ny = 40
    s, x0, y0 = 50.0, -0.4, -0.4
    xc = x0 + (np.arange(nx) + 0.5) / s
    H = np.repeat((0.02 * xc)[None, :], ny, 0).astype(np.float32)
    hf = _table(H, s, x0, y0)
    p = W.Params(hf_bilinear=True, mu=math.inf)
    ow = scene(box_morph(), [0.0, 0.0, 0.05, 1, 0, 0, 0], params=p, hf=hf)
    st = ow.init_state(0)
    ow.run(0, st, 3000)
    assert st[O.FLAGS] == 0
    P = ow.points(0, st)
    low = P[P[:, 2] < st[O.C_ + 2]]
    # the bottom corners rest just below the plane z = 0.02 x
    gaps = low[:, 2] - 0.02 * low[:, 0]
    assert np.all(gaps < 0) and np.all(gaps > -2e-3), gaps
    assert np.linalg.norm(st[O.V_:O.V_ + 3]) < 1e-3


def _arm_in_flight(params):
    """A box torso with one hinged arm, 5 m above flat ground (no contact), the
    arm commanded sin(2 pi t) rad."""
    pts = [[sx * 0.1, sy * 0.05, sz * 0.025, 0.125] for sx in (-1, 1) for sy in (-1, 1)
           for sz in (-1, 1)] + [[0.2, 0, 0, 0.1], [0.3, 0, 0, 0.1]]
    joint = np.zeros((2, 8), np.float32)
    joint[1] = [0.1, 0, 0, 0, 1, 0, -10, 10]
    arm = W.Morph(points=np.array(pts, np.float32), pt_link=np.array([0] * 8 + [1, 1], np.int32),
                  parent=np.array([-1, 0], np.int32), joint=joint, name="arm")
    w = W.Workload(params=params, hf=W.flat_ground(), morphs=[arm],
                   inst_morph=np.zeros(1, np.int32),
                   ctrl=[np.array([[1.0, 1.0, 0.0]], np.float32)],
                   pose=np.array([[0, 0, 5.0, 1, 0, 0, 0]], np.float32))
    return O.OracleWorld(w)


@pytest.mark.parametrize("K", [1, 8])
def test_joint_rate_limit_ramps_at_the_limit(K):
    """A command sin(2 pi t) rad rises faster than 1 rad/s near t = 0, so a joint
    limited to 1 rad/s ramps by exactly r K dt per update: after frames 0..99
    it has moved on every update after the first (t = 0, command 0)."""
    ow = _arm_in_flight(W.Params(K=K, max_joint_rate=1.0))
    st = ow.init_state(0)
    ow.run(0, st, 100)
    d = 1.0 * K * 1e-3
    moves = len(range(K, 100, K))
    q, qp = st[O.HDR], st[O.HDR + 1]
    assert abs(q - moves * d) < 1e-12 and abs((q - qp) - d) < 1e-12
    # unlimited, the joint follows the command itself
    ow0 = _arm_in_flight(W.Params(K=K))
    st0 = ow0.init_state(0)
    ow0.run(0, st0, 100)
    assert abs(st0[O.HDR] - math.sin(2 * math.pi * (moves * K) * 1e-3)) < 1e-12


def test_joint_rate_limit_bounds_every_update_and_vanishes_when_loose():
    """On hexapods on the terrain: every update moves a joint by at most r K dt
    and some updates move one by exactly that; a limit that never binds (1e6 rad/s), zero and
    +inf all give the unlimited trajectory bit for bit."""
    w = W.hexapod_batch(2, seed=8)
    ref = O.OracleWorld(w)
    st_ref = ref.init_state(1)
    ref.run(1, st_ref, 300)
    for r in (0.0, math.inf, 1e6):
        w.params.max_joint_rate = r
        ow = O.OracleWorld(w)
        st = ow.init_state(1)
        ow.run(1, st, 300)
        assert np.array_equal(st, st_ref), r
    w.params.max_joint_rate = 0.5
    w.params.K = 4
    ow = O.OracleWorld(w)
    st = ow.init_state(1)
    J = w.morphs[0].n_links - 1
    d = 0.5 * 4 * 1e-3
    binding = 0
    for n in range(300):
        before = st.copy()
        ow.step(1, st)
        if n % 4 == 0:
            dq = st[O.HDR:O.HDR + J] - before[O.HDR:O.HDR + J]
            assert np.all(np.abs(dq) <= d * (1 + 1e-12))
            binding += int(np.sum(np.abs(dq) > d * (1 - 1e-12)))
    assert binding > 0
