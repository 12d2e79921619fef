"""Pins of the oracle's log of fragile decisions and of its flips.

A fragile decision is an integer outcome of the step decided by floating point
that a change far below the parity tolerances could turn: a height-map look-up
next to a cell edge (Sec. III-A: the coordinates scaled to integer indices), a
contact test at almost zero depth, the spread test of the friction fit and the
comparison with the maximum static friction (Sec. III-C). The GPU parity checks
use the log to name the decision a float32 frame took the other way, and the
flip to verify it. These pins fix what is logged and what a flip changes, on
scenes whose outcome is known in closed form.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2411_05799_amd import workloads as W

G0 = 9.81
HALF_Z = float(np.float32(0.05 / 2))


def one_body(points, pose, params=None, hf=None):
    pts = np.asarray(points, np.float32)
    m = W.Morph(points=pts, pt_link=np.zeros(len(pts), np.int32),
                parent=np.array([-1], np.int32), joint=np.zeros((1, 8), np.float32), name="body")
    w = W.Workload(params=params or W.Params(), hf=hf or W.flat_ground(), morphs=[m],
                   inst_morph=np.zeros(1, np.int32), ctrl=[np.zeros((0, 3), np.float32)],
                   pose=np.asarray(pose, np.float32)[None, :])
    return O.OracleWorld(w)


def box_points(mass=1.0, lx=0.2, ly=0.1, lz=0.05):
    return [[sx * lx / 2, sy * ly / 2, sz * lz / 2, mass / 8]
            for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]


def step_map():
    """Two cells of 0.1 m along x (edge at x = 0.1), heights 1 cm and 3 cm."""
    H = np.array([[0.01, 0.03]], np.float32)
    return W.Heightfield(nx=2, ny=1, s=10.0, x0=0.0, y0=0.0, H=H)


def test_margins_zero_is_the_plain_step():
    """With no margin and no flip, step_ex is the plain step bit for bit (a
    hexapod walking on the terrain, 300 frames), and logs nothing."""
    w = W.hexapod_batch(2, seed=3, hf=W.octave_terrain(3), spread=0.5)
    ow = O.OracleWorld(w)
    for i in range(2):
        a = ow.init_state(i)
        b = a.copy()
        for _ in range(300):
            ow.step(i, a)
            assert ow.step_ex(i, b) == []
        np.testing.assert_array_equal(a, b)


def test_logging_does_not_change_the_step():
    """Margins without flips only log: the state is the plain step's bit for bit."""
    w = W.hexapod_batch(2, seed=4, hf=W.octave_terrain(3), spread=0.5)
    ow = O.OracleWorld(w)
    seen = 0
    for i in range(2):
        a = ow.init_state(i)
        b = a.copy()
        for _ in range(300):
            ow.step(i, a)
            seen += len(ow.step_ex(i, b, margin_m=1e-3, margin_rel=1e-3))
        np.testing.assert_array_equal(a, b)
    assert seen > 0   # 1 mm margins on a 2 cm grid: feet sit near edges often


def test_edge_lookup_logged_and_flipped():
    """A single mass point 1e-7 m left of the cell edge x = 0.1, 5 mm into the
    lower (1 cm) cell: its look-ups (S1 at P^n, S5 at P*, and the telemetry's
    under the torso origin, which for one point is the point) are logged at that
    distance; the normal force is k_n * 5 mm, and 25 mm (the other cell's depth)
    with the S1 look-up flipped; the flipped telemetry look-up reads 2 cm more
    ground."""
    p = W.Params()
    x = 0.1 - 1e-7
    ow = one_body([[0, 0, 0, 1.0]], [x, 0.05, 0.005, 1, 0, 0, 0], params=p, hf=step_map())
    st = ow.init_state(0)
    x32 = float(np.float32(x))                 # the pose is handed over in float32
    log, d = ow.step_ex(0, st.copy(), margin_m=1e-6, diag=True)
    kinds = {(s, k, kind) for s, k, kind, _ in log}
    assert kinds == {(O.FR_S1, 0, O.FK_EDGE_X), (O.FR_S5, 0, O.FK_EDGE_X),
                     (O.FR_S9, -1, O.FK_EDGE_X)}
    for _, _, _, dist in log:
        assert abs(dist - (0.1 - x32)) < 1e-12
    z = float(np.float32(0.005))
    assert abs(d[O.D_FN] - p.k_n * (0.01 - z)) < 1e-9 * p.k_n
    _, d2 = ow.step_ex(0, st.copy(), margin_m=1e-6, flips=[(O.FR_S1, 0, O.FK_EDGE_X)], diag=True)
    assert abs(d2[O.D_FN] - p.k_n * (float(np.float32(0.03)) - z)) < 1e-9 * p.k_n
    a, b = st.copy(), st.copy()
    ow.step_ex(0, a, margin_m=1e-6)
    ow.step_ex(0, b, margin_m=1e-6, flips=[(O.FR_S9, -1, O.FK_EDGE_X)])
    dh = float(np.float32(0.03)) - float(np.float32(0.01))
    assert abs((a[O.TELE] - b[O.TELE]) - dh) < 1e-15
    # far from the edge nothing is logged; above both cells the detection
    # look-ups are not (only the telemetry's, which reads the ground anyway)
    ow2 = one_body([[0, 0, 0, 1.0]], [0.05, 0.05, 0.005, 1, 0, 0, 0], params=p, hf=step_map())
    assert ow2.step_ex(0, ow2.init_state(0), margin_m=1e-6) == []
    ow3 = one_body([[0, 0, 0, 1.0]], [x, 0.05, 0.05, 1, 0, 0, 0], params=p, hf=step_map())
    assert [e[0] for e in ow3.step_ex(0, ow3.init_state(0), margin_m=1e-6)] == [O.FR_S9]


def test_edge_below_lower_cell_only_matters_when_heights_differ():
    """Equal heights on both sides: the look-up's cell cannot change anything, so
    it is not logged even right at the edge."""
    H = np.array([[0.02, 0.02]], np.float32)
    hf = W.Heightfield(nx=2, ny=1, s=10.0, x0=0.0, y0=0.0, H=H)
    ow = one_body([[0, 0, 0, 1.0]], [0.1 - 1e-9, 0.05, 0.0, 1, 0, 0, 0], hf=hf)
    assert ow.step_ex(0, ow.init_state(0), margin_m=1e-6) == []


def test_contact_sign_logged_and_flipped():
    """A box whose bottom corners are 1e-9 m into the plane: four contacts at
    depth 1e-9 are logged at S1; flipping one leaves three contacts."""
    ow = one_body(box_points(), [0.0, 0.0, 0.0, 1, 0, 0, 0])
    st = ow.init_state(0)
    st[O.C_ + 2] = HALF_Z - 1e-9
    log, d = ow.step_ex(0, st.copy(), margin_m=1e-6, diag=True)
    s1 = [e for e in log if e[0] == O.FR_S1]
    assert len(s1) == 4 and all(e[2] == O.FK_CONTACT and abs(e[3] - 1e-9) < 1e-15 for e in s1)
    assert d[O.D_NC] == 4
    k = s1[0][1]
    _, d2 = ow.step_ex(0, st.copy(), margin_m=1e-6, flips=[(O.FR_S1, k, O.FK_CONTACT)],
                       diag=True)
    assert d2[O.D_NC] == 3


def test_spread_test_logged_and_flipped():
    """Two mass points 2e-4 m apart resting on the plane and spinning about z:
    their spread is W eps^2 (the rotation test of eqs. 4-6 sits on its
    threshold), so it is logged; the translation-only branch leaves the spin,
    the full fit stops it."""
    p = W.Params()
    e = 1e-4
    ow = one_body([[-e, 0, 0, 0.5], [e, 0, 0, 0.5]], [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_ + 2] = -G0 / (2 * p.k_n)          # resting depth of two points sharing 1 kg
    st[O.W_ + 2] = 1.0
    log = ow.step_ex(0, st.copy(), margin_rel=1e-3)
    assert [(s, k, kind) for s, k, kind, _ in log] == [(O.FR_FIT, -1, O.FK_SPREAD)]
    a = st.copy()
    ow.step_ex(0, a, margin_rel=1e-3)
    b = st.copy()
    ow.step_ex(0, b, margin_rel=1e-3, flips=[(O.FR_FIT, -1, O.FK_SPREAD)])
    spins = sorted([abs(a[O.W_ + 2]), abs(b[O.W_ + 2])])
    assert spins[0] < 1e-6 and abs(spins[1] - 1.0) < 1e-9


def test_cap_logged_and_flip_changes_only_the_slip_count():
    """On the incline exactly at tan(theta) = mu the friction estimate equals
    mu F_N: the comparison is logged, and flipping it changes the slipping-frame
    count by one and nothing else (the cap factor is 1 on both sides)."""
    mu = 0.5
    theta = math.atan(mu)
    p = W.Params(g=(G0 * math.sin(theta), 0.0, -G0 * math.cos(theta)), mu=mu)
    d_eq = G0 * math.cos(theta) / (4 * p.k_n)
    ow = one_body(box_points(), [0.0, 0.0, 0.0, 1, 0, 0, 0], params=p)
    st = ow.init_state(0)
    st[O.C_:O.C_ + 3] = [0.0, 0.0, HALF_Z - d_eq]
    a, b = st.copy(), st.copy()
    log = ow.step_ex(0, a, margin_rel=1e-6)
    assert (O.FR_FIT, -1, O.FK_CAP) in [(s, k, kind) for s, k, kind, _ in log]
    ow.step_ex(0, b, margin_rel=1e-6, flips=[(O.FR_FIT, -1, O.FK_CAP)])
    assert abs(a[O.TELE + 2] - b[O.TELE + 2]) == 1.0
    keep = np.ones(a.size, bool)
    keep[O.TELE + 2] = False
    np.testing.assert_array_equal(a[keep], b[keep])
