"""Shared helpers of the parity tests: moving states between the FP64 oracle and
the GPU world, and the error measures the tolerances are stated in."""
import math

import numpy as np

from oracle import oracle as O
from paper_2411_05799_amd import native as N

# tolerances of the GPU FP32 path against the FP64 oracle over 200-frame windows
POS_TOL = 1e-4     # m: CoG and every mass point
ANG_TOL = 1e-3     # rad: joint angles and torso orientation
STAT_TOL = 0.02    # relative: long-horizon statistics


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def round_state(st):
    """The oracle state rounded to float32 and back (the window's start state)."""
    out = st.copy()
    out[:O.TELE] = st[:O.TELE].astype(np.float32).astype(np.float64)
    out[O.HDR:] = st[O.HDR:].astype(np.float32).astype(np.float64)
    return out


def write_states(gw, idx, states, J_of):
    """Overwrite instances idx of the GPU world with oracle states (float32)."""
    body = gw.read_state(N.F_BODY)
    q = gw.read_state(N.F_JOINT)
    qp = gw.read_state(N.F_JOINT_PREV)
    step = gw.read_state(N.F_STEP)
    flags = gw.read_state(N.F_FLAGS)
    for i, st in zip(idx, states):
        J = J_of(i)
        body[:, i] = st[:13].astype(np.float32)
        q[:J, i] = st[O.HDR:O.HDR + J].astype(np.float32)
        qp[:J, i] = st[O.HDR + J:O.HDR + 2 * J].astype(np.float32)
        step[i] = int(st[O.STEP])
        flags[i] = int(st[O.FLAGS])
    gw.write_state(N.F_BODY, body)
    gw.write_state(N.F_JOINT, q)
    gw.write_state(N.F_JOINT_PREV, qp)
    gw.write_state(N.F_STEP, step)
    gw.write_state(N.F_FLAGS, flags)


def read_states(gw, idx, J_of):
    """GPU states of instances idx as oracle-layout float64 vectors."""
    body = gw.read_state(N.F_BODY)
    q = gw.read_state(N.F_JOINT)
    qp = gw.read_state(N.F_JOINT_PREV)
    step = gw.read_state(N.F_STEP)
    flags = gw.read_state(N.F_FLAGS)
    tele = gw.read_state(N.F_TELE)
    out = []
    for i in idx:
        J = J_of(i)
        st = np.zeros(O.HDR + 2 * J)
        st[:13] = body[:, i]
        st[O.STEP] = step[i]
        st[O.FLAGS] = flags[i]
        st[O.TELE:O.TELE + 4] = tele[:, i]
        st[O.HDR:O.HDR + J] = q[:J, i]
        st[O.HDR + J:] = qp[:J, i]
        out.append(st)
    return out


def quat_angle(q1, q2):
    """Geodesic angle between two unit quaternions."""
    d = abs(float(np.dot(q1, q2)) / (np.linalg.norm(q1) * np.linalg.norm(q2)))
    return 2.0 * math.acos(min(1.0, d))


class WindowStats:
    def __init__(self):
        self.cog = 0.0
        self.pts = 0.0
        self.joint = 0.0
        self.orient = 0.0
        self.start = None      # oracle state at the window start (rounded to float32)
        self.spread = None     # oracle ensemble spread, filled in for windows off tolerance

    def update(self, ref, got, Pref=None, Pgot=None, J=0):
        self.cog = max(self.cog, float(np.abs(ref[:3] - got[:3]).max()))
        self.orient = max(self.orient, quat_angle(ref[3:7], got[3:7]))
        if J:
            self.joint = max(self.joint, float(np.abs(ref[O.HDR:O.HDR + J]
                                                      - got[O.HDR:O.HDR + J]).max()))
        if Pref is not None:
            self.pts = max(self.pts, float(np.abs(Pref - Pgot).max()))

    def ok(self):
        return (self.cog <= POS_TOL and self.pts <= POS_TOL and self.joint <= ANG_TOL
                and self.orient <= ANG_TOL)

    def __repr__(self):
        return (f"cog {self.cog:.2e} m, points {self.pts:.2e} m, joints {self.joint:.2e} rad, "
                f"orientation {self.orient:.2e} rad")


def run_windows(ow, gw, idx, starts, length=200, every=20, check_points=True):
    """For each window start s: the oracle trajectory at frame s, rounded to FP32,
    is written to the GPU; both advance `length` frames and are compared every
    `every` frames. Returns one WindowStats per (start, instance)."""
    J_of = lambda i: ow.morph_of(i).n_joints
    traj = {i: ow.init_state(i) for i in idx}
    pos = {i: 0 for i in idx}
    results = []
    for s in starts:
        for i in idx:
            ow.run(i, traj[i], s - pos[i])
            pos[i] = s
        start = {i: round_state(traj[i]) for i in idx}
        write_states(gw, idx, [start[i] for i in idx], J_of)
        refs = {i: start[i].copy() for i in idx}
        stats = {i: WindowStats() for i in idx}
        for i in idx:
            stats[i].start = start[i].copy()
        for k in range(0, length, every):
            for i in idx:
                ow.run(i, refs[i], every)
            gw.step_n(every)
            got = read_states(gw, idx, J_of)
            P = gw.read_points() if check_points else None
            for i, g in zip(idx, got):
                n_pts = ow.morph_of(i).n_points
                Pref = ow.points(i, refs[i]) if check_points else None
                Pgot = P[i, :n_pts] if check_points else None
                stats[i].update(refs[i], g, Pref, Pgot, J_of(i))
        results += [(s, i, stats[i]) for i in idx]
    return results


# Relative size of the per-frame perturbation of the noisy oracle ensemble. From
# identical start states, one frame of the float32 GPU path deviates from the
# oracle by ~2^-25 relative in position and orientation, and by 2^-14..2^-18
# relative in velocity and angular velocity (stiff contact turns 1e-8 m of
# position rounding into ~1e-6 m/s); the ensemble perturbs every component by
# up to 2^-20 per frame.
NOISE_REL = 2.0 ** -20


def _noisy_run(ow, i, st, n, rng, J):
    """n oracle frames, each followed by a relative perturbation (uniform in
    +-NOISE_REL) of the CoG, orientation, velocities and joint angles."""
    for _ in range(n):
        ow.step(i, st)
        for a, b in ((0, 13), (O.HDR, O.HDR + 2 * J)):
            st[a:b] *= 1.0 + rng.uniform(-1.0, 1.0, b - a) * NOISE_REL


def ensemble_spread(ow, i, start, members=4, length=200, every=20, seed=0):
    """Largest deviation (CoG or any mass point, m; orientation, rad) of oracle
    runs with float32-scale noise from the noiseless oracle over one window: how
    well the FP64 step itself determines this window at float32 resolution."""
    J = ow.morph_of(i).n_joints
    rng = np.random.default_rng(seed)
    ref = start.copy()
    mem = [start.copy() for _ in range(members)]
    pos, ang = 0.0, 0.0
    for _ in range(0, length, every):
        ow.run(i, ref, every)
        Pr = ow.points(i, ref)
        for m in mem:
            _noisy_run(ow, i, m, every, rng, J)
            pos = max(pos, float(np.abs(ow.points(i, m) - Pr).max()),
                      float(np.abs(m[:3] - ref[:3]).max()))
            ang = max(ang, quat_angle(m[3:7], ref[3:7]))
    return pos, ang


SPREAD_FACTOR = 3.0
MAX_ILL_FRACTION = 0.50


def judge_windows(ow, results):
    """A window passes if it is within POS_TOL / ANG_TOL, or, when the FP64 oracle
    itself is not determined to that tolerance at float32 resolution (its noisy
    ensemble spreads wider), if the GPU stays within SPREAD_FACTOR times that
    spread. Returns (failures, ill-conditioned windows)."""
    bad, ill = [], []
    for s, i, st in results:
        if st.ok():
            continue
        st.spread = ensemble_spread(ow, i, st.start)
        pos_sp, ang_sp = st.spread
        pos_err = max(st.cog, st.pts)
        ang_err = max(st.joint, st.orient)
        well_pos = pos_err <= POS_TOL or pos_err <= SPREAD_FACTOR * pos_sp
        well_ang = ang_err <= ANG_TOL or ang_err <= SPREAD_FACTOR * ang_sp
        if well_pos and well_ang and (pos_sp > POS_TOL / SPREAD_FACTOR
                                      or ang_sp > ANG_TOL / SPREAD_FACTOR):
            ill.append((s, i, st))
        else:
            bad.append((s, i, st))
    return bad, ill
