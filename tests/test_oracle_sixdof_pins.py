"""Pins of the oracle's six-degree-of-freedom friction fit (the refinement that
closes Sec. III-C: rotations about the other two axes as well): the linear
algebra against textbook routines and exact rigid data (Kabsch), the reduction
to the ground-plane fit of eqs. (4)-(6), origin covariance, the degenerate
sets, and the step with the option on (rest, incline threshold, roll stop).
CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_05799_amd import workloads as W

from test_oracle_pins import G0, HALF_Z, box_morph, energy, kabsch, scene


def rotvec(R):
    """Rotation vector of a rotation matrix (textbook log map, angle < pi)."""
    c = max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0))
    ang = math.acos(c)
    v = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    if ang < 1e-12:
        return 0.5 * v
    return ang / (2.0 * math.sin(ang)) * v


def rot(phi):
    """Rotation matrix of a rotation vector (Rodrigues)."""
    a = float(np.linalg.norm(phi))
    if a == 0.0:
        return np.eye(3)
    k = phi / a
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(a) * K + (1 - math.cos(a)) * K @ K


# ----------------------------------------------------------------------------
# the smallest eigenvalue of the spread tensor
# ----------------------------------------------------------------------------

def test_sym3_min_eig_matches_eigvalsh():
    rng = np.random.default_rng(5)
    for _ in range(200):
        B = rng.normal(size=(3, 3))
        A = B + B.T
        ref = np.linalg.eigvalsh(A)[0]
        assert abs(O.sym3_min_eig(A) - ref) <= 1e-12 * max(1.0, np.abs(A).max())
    # special cases: a multiple of the identity, a repeated pair, rank one, zero
    assert O.sym3_min_eig(2.5 * np.eye(3)) == 2.5
    assert abs(O.sym3_min_eig(np.diag([3.0, 1.0, 1.0])) - 1.0) < 1e-14
    assert abs(O.sym3_min_eig(np.outer([1.0, 2.0, 2.0], [1.0, 2.0, 2.0]))) < 1e-13
    assert O.sym3_min_eig(np.zeros((3, 3))) == 0.0


# ----------------------------------------------------------------------------
# the fit itself
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("scale", [1e-6, 1e-4, 1e-2])
def test_fit_of_rigid_data_is_kabsch_to_second_order(scale):
    """Points carried by an exact rigid motion (R, t): the first-order fit
    recovers Kabsch's rotation vector and translation up to the neglected
    second-order term of the rotation (|phi|^2 relative)."""
    rng = np.random.default_rng(int(-math.log10(scale)))
    src = rng.normal(size=(12, 3)) * 0.1
    phi = rng.normal(size=3) * scale
    t = rng.normal(size=3) * scale * 0.1
    dst = src @ rot(phi).T + t
    Rk, tk = kabsch(src, dst)
    np.testing.assert_allclose(Rk, rot(phi), atol=1e-13)        # Kabsch is exact
    a, k = O.lsq6(src, dst)
    assert k == 6
    pk = rotvec(Rk)
    err = np.linalg.norm(a[3:] - pk)
    assert err <= 4 * np.linalg.norm(pk) ** 2 + 1e-15
    # the displacement of the origin: t to the same order (points ~0.1 m out)
    assert np.linalg.norm(a[:3] - tk) <= 4 * 0.3 * np.linalg.norm(pk) ** 2 + 1e-15


def test_fit_equals_lstsq_of_the_linearized_residuals():
    """The 6x6 normal equations against numpy's least squares on the stacked
    residual rows, with weights."""
    rng = np.random.default_rng(2)
    src = rng.normal(size=(9, 3)) * 0.1
    dst = src + rng.normal(size=(9, 3)) * 1e-3
    w = rng.uniform(0.1, 2.0, 9)
    rows, rhs = [], []
    for x, y, wi in zip(src, dst, w):
        for c in range(3):
            g = np.zeros(6)
            g[c] = 1.0
            for k in range(3):
                e = np.zeros(3)
                e[k] = 1.0
                g[3 + k] = np.cross(e, x)[c]
            rows.append(math.sqrt(wi) * g)
            rhs.append(math.sqrt(wi) * (y[c] - x[c]))
    ref = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
    a, k = O.lsq6(src, dst, weights=w)
    assert k == 6
    np.testing.assert_allclose(a, ref, rtol=1e-10, atol=1e-15)


def test_pure_translation_is_exact():
    rng = np.random.default_rng(3)
    src = rng.normal(size=(6, 3)) * 0.1
    t = np.array([2e-4, -1e-4, 3e-5])
    a, k = O.lsq6(src, src + t)
    assert k == 6
    np.testing.assert_allclose(a[:3], t, atol=1e-17)
    assert np.abs(a[3:]).max() < 1e-15


@pytest.mark.parametrize("h", [0.0, -0.12, 0.3])
@pytest.mark.parametrize("weighted", [False, True])
def test_level_set_with_horizontal_slips_reduces_to_the_ground_plane_fit(h, weighted):
    """Contact points at one height h and slips in the ground plane: no roll,
    pitch or vertical displacement, and (a1, a2, a3) of eqs. (4)-(6)."""
    rng = np.random.default_rng(7)
    n = 8
    xy = rng.normal(size=(n, 2)) * 0.1
    d = rng.normal(size=(n, 2)) * 1e-4
    src = np.c_[xy, np.full(n, h)]
    dst = np.c_[xy + d, np.full(n, h)]
    w = rng.uniform(0.2, 3.0, n) if weighted else None
    a, k = O.lsq6(src, dst, weights=w)
    a3, k3 = O.lsq(xy, xy + d, weights=w)
    assert k == 6 and k3 == 3
    scale = np.abs(a3).max()
    np.testing.assert_allclose(a[[0, 1, 5]], a3, rtol=1e-9, atol=1e-13 * scale)
    assert np.abs(a[2:5]).max() <= 1e-12 * scale


def test_fit_is_covariant_in_its_origin():
    """Shifting every coordinate by o keeps the rotation and moves the
    displacement to the new origin: a' = a + th x o."""
    rng = np.random.default_rng(11)
    src = rng.normal(size=(7, 3)) * 0.1
    dst = src + rng.normal(size=(7, 3)) * 1e-4
    o = np.array([0.3, -0.2, 0.05])
    a, _ = O.lsq6(src, dst)
    b, _ = O.lsq6(src - o, dst - o)
    np.testing.assert_allclose(b[3:], a[3:], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(b[:3], a[:3] + np.cross(a[3:], o), rtol=1e-9, atol=1e-15)


def test_degenerate_sets_fall_back_to_the_ground_plane_fit():
    """A set on one line (rotation about it undetermined), one within 1 mm of a
    line over 20 cm (spread ratio under 1e-3) and a single point: the
    ground-plane fit on x, y with the mean vertical slip; no roll, pitch. 1 cm
    off the line the rotation is fitted in 3-D."""
    rng = np.random.default_rng(13)
    u = np.array([0.6, 0.8, 0.0])
    s = np.linspace(-0.1, 0.1, 5)
    src = np.outer(s, u) + np.array([0.0, 0.0, -0.1])
    dst = src + rng.normal(size=(5, 3)) * 1e-4
    a, k = O.lsq6(src, dst)
    a3, k3 = O.lsq(src[:, :2], dst[:, :2])
    assert k == k3 == 3
    np.testing.assert_allclose(a[[0, 1, 5]], a3, rtol=1e-12, atol=1e-18)
    assert abs(a[2] - (dst - src)[:, 2].mean()) < 1e-18
    assert a[3] == 0.0 and a[4] == 0.0
    # nearly on a line: 1 mm off it over 20 cm, spread ratio below 1e-3
    near = src + np.outer(np.array([1, -1, 1, -1, 1]) * 1e-3, [0.0, 0.0, 1.0])
    S = sum(np.dot(e, e) * np.eye(3) - np.outer(e, e) for e in near - near.mean(0))
    assert O.sym3_min_eig(S) < 1e-3 * np.trace(S) and O.sym3_min_eig(S) > 5 * 1e-8
    a, k = O.lsq6(near, near + (dst - src))
    assert k == 3 and a[3] == 0.0 and a[4] == 0.0
    wide = src + np.outer(np.array([1, -1, 1, -1, 1]) * 1e-2, [0.0, 0.0, 1.0])
    a, k = O.lsq6(wide, wide + (dst - src))
    assert k == 6
    one = np.array([[0.1, 0.2, -0.1]])
    a, k = O.lsq6(one, one + [1e-4, -2e-4, 3e-4])
    assert k == 2
    np.testing.assert_allclose(a, [1e-4, -2e-4, 3e-4, 0, 0, 0], atol=1e-18)
    a, k = O.lsq6(np.zeros((0, 3)), np.zeros((0, 3)))
    assert k == 0 and not a.any()


# ----------------------------------------------------------------------------
# the step with the option on
# ----------------------------------------------------------------------------

def p6(**kw):
    return W.Params(friction_6dof=True, **kw)


def test_six_dof_with_force_weighting_is_refused():
    """The two refinements are not combined: with the force on points along one
    line, a point of near-zero force would decide the roll about that line."""
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0],
               params=W.Params(friction_6dof=True, friction_weighting=True))
    st = ow.init_state(0)
    with pytest.raises(AssertionError):
        ow.step(0, st)
    with pytest.raises(AssertionError):
        ow.run_batch([st], 3)


def test_free_flight_is_the_plain_step():
    """No contact, no friction set: bit for bit the ground-plane step."""
    box = box_morph()
    a = scene(box, [0.0, 0.0, 1.0, 0.9, 0.1, 0.3, 0.2], params=W.Params())
    b = scene(box, [0.0, 0.0, 1.0, 0.9, 0.1, 0.3, 0.2], params=p6())
    sa, sb = a.init_state(0), b.init_state(0)
    sa[O.W_:O.W_ + 3] = sb[O.W_:O.W_ + 3] = [1.0, -2.0, 0.5]
    a.run(0, sa, 200)
    b.run(0, sb, 200)
    np.testing.assert_array_equal(sa, sb)


def test_rest_is_an_equilibrium_with_six_dof():
    p = p6()
    mass = 1.5
    d_eq = mass * G0 / (4 * p.k_n)
    ow = scene(box_morph(mass=mass), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_ + 2] = HALF_Z - d_eq
    c0 = st[:13].copy()
    E0 = energy(ow, st, p)
    ow.run(0, st, 5000)
    assert abs(energy(ow, st, p) - E0) <= 1e-12 * abs(E0)
    np.testing.assert_allclose(st[:13], c0, atol=1e-12)


def test_landing_has_no_energy_gain_and_the_contact_set_stops():
    """Dropped flat: the first frame with a friction set stops its vertical
    motion (3-D static friction holds the contact points in every direction),
    so the box comes to rest at once, at a depth above the penalty
    equilibrium, and stays there."""
    p = p6()
    ow = scene(box_morph(), [0.0, 0.0, HALF_Z + 0.02, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    E0 = energy(ow, st, p)
    ns = []
    for _ in range(400):
        d = ow.step(0, st, diag=True)
        ns.append(d[O.D_NS])
        assert energy(ow, st, p) <= E0 + 1e-9
    first = ns.index(4)
    assert abs(st[O.V_ + 2]) < 1e-12
    z = st[O.C_ + 2]
    ow.run(0, st, 500)
    assert abs(st[O.C_ + 2] - z) < 1e-12
    d_eq = 1.0 * G0 / (4 * p.k_n)
    assert HALF_Z - d_eq < z < HALF_Z          # in contact, shallower than at rest
    assert first < 400


@pytest.mark.parametrize("side", [-1, +1])
def test_incline_threshold_with_six_dof(side):
    """At the penalty rest depth the contact set has no vertical slip, so the
    incline behaves as with the ground-plane fit: sticks iff tan(theta) <= mu,
    else slides with x_n = g (sin - mu cos) dt^2 n (n+1) / 2."""
    mu = 0.5
    theta = math.atan(mu) * (1 + side * 1e-3)
    p = p6(g=(G0 * math.sin(theta), 0.0, -G0 * math.cos(theta)), mu=mu)
    d_eq = G0 * math.cos(theta) / (4 * p.k_n)
    ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
    n = 5000
    ow.run(0, st, n)
    dx = st[O.C_]
    if side < 0:
        assert abs(dx) < 1e-11
    else:
        xn = G0 * (math.sin(theta) - mu * math.cos(theta)) * p.dt ** 2 * n * (n + 1) / 2
        assert abs(dx - xn) <= 1e-8 * xn
    np.testing.assert_allclose(st[O.Q_:O.Q_ + 4], [1, 0, 0, 0], atol=1e-12)


def test_rolling_box_is_stopped_only_with_six_dof():
    """A resting box given a roll rate about x: its contact points move up and
    down (and, 2.5 cm below the CoG, sideways by dt w_x HALF_Z: an implied
    friction force well under mu F_N at this rate), the six-degree fit finds
    the roll (sin of dt w_x) and the correction removes it; the ground-plane
    fit only removes the sideways slip and leaves the roll."""
    w0 = 0.1
    out = {}
    for six in (False, True):
        p = W.Params(friction_6dof=six)
        d_eq = G0 / (4 * p.k_n)
        ow = scene(box_morph(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
        st = ow.init_state(0)
        st[O.C_ + 2] = HALF_Z - d_eq
        st[O.W_] = w0
        d = ow.step(0, st, diag=True)
        out[six] = (st.copy(), d)
    st6, d6 = out[True]
    assert d6[O.D_NS] == 4 and d6[O.D_LAMBDA] == 1.0
    # the trial roll is dt w1, w1 a little below w0 (the normal forces' torque
    # of the frame opposes it); the correction removes it to the fit's second
    # order (|dt w|^2 / dt = 1e-5 rad/s)
    assert 0.9 * w0 * 1e-3 < d6[O.D_A6 + 3] <= w0 * 1e-3
    assert abs(st6[O.W_]) < 1e-5
    st3, _ = out[False]
    assert abs(st3[O.W_]) > 0.05


def test_six_dof_conditioning_test_logged_and_flipped():
    """Four resting points at (+-5 cm, +-e) with e chosen so that the spread
    tensor's smallest eigenvalue 4 e^2 is 1e-3 of its trace 8 (0.05^2 + e^2)
    (the conditioning bound, above W eps^2): the test is logged as the fit's
    fragile decision at point -2; with a roll rate about x the full fit stops
    the roll and the ground-plane branch leaves it."""
    from test_oracle_fragile_pins import one_body
    p = p6()
    e = math.sqrt(2e-3 * 0.05 ** 2 / (1 - 2e-3))
    pts = [[sx * 0.05, sy * e, 0.0, 0.25] for sx in (-1, 1) for sy in (-1, 1)]
    ow = one_body(pts, [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_ + 2] = -G0 / (4 * p.k_n)
    st[O.W_] = 1.0
    log = ow.step_ex(0, st.copy(), margin_rel=1e-3)
    assert (O.FR_FIT, -2, O.FK_SPREAD) in [(s, k, kind) for s, k, kind, _ in log]
    a, b = st.copy(), st.copy()
    ow.step_ex(0, a, margin_rel=1e-3)
    ow.step_ex(0, b, margin_rel=1e-3, flips=[(O.FR_FIT, -2, O.FK_SPREAD)])
    rolls = sorted([abs(a[O.W_]), abs(b[O.W_])])
    assert rolls[0] < 1e-3 and rolls[1] > 0.9
