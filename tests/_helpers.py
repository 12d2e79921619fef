"""Shared helpers of the parity tests: moving states between the FP64 oracle and
the GPU world, and the two checks the tolerances are stated in.

Window check. From an oracle state rounded to float32 and written to the GPU,
both advance `length` frames; every frame the CoG, every mass point (the FP64
positions of each side's state), the joint angles and the torso orientation
are compared: 1e-4 m and 1e-3 rad.

Frame check. Every GPU frame is also compared with ONE oracle frame taken from
the GPU's own state before it (read back exactly; the oracle steps it in
FP64). This isolates the float32 step from the chaos of contact dynamics: the
two differ by float32 rounding only (FRAME_TOL), unless the frame is
ill-conditioned or took one of the step's fragile decisions (a look-up within
FRAGILE_MARGIN_M of a cell edge, a contact test at near-zero depth, a fit
threshold) the other way. For a frame beyond FRAME_TOL:
  * conditioning: the oracle frame is taken again from ENSEMBLE copies of its
    inputs perturbed by one float32 rounding (the state, 2^-23 relative per
    component, and the controller parameters, one ulp); the bound of each
    quantity grows by SENS times the spread of those copies (how far
    float32-sized input changes alone move this frame's result);
  * fragile decisions: the oracle's log of the frame's fragile decisions is
    searched; the frame is explained if the oracle frame with one (or two) of
    them flipped matches the GPU frame within that bound.
A frame that matches neither way is a failure, whatever its window does.

Verdict of a window: within the window tolerances, or beyond them but made of
verified frames only (float32 rounding amplified by the contact dynamics, or a
flipped fragile decision, named in the report); at most
MAX_ATTRIBUTED_FRACTION of a test's windows may be of the second kind.
"""
import itertools
import math

import numpy as np

from oracle import oracle as O
from paper_2411_05799_amd import native as N

# tolerances of the GPU FP32 path against the FP64 oracle over 200-frame windows
POS_TOL = 1e-4     # m: CoG and every mass point
ANG_TOL = 1e-3     # rad: joint angles and torso orientation
STAT_TOL = 0.02    # relative: long-horizon statistics
MAX_ATTRIBUTED_FRACTION = 0.10

# One float32 frame from a float32 state against the FP64 frame from the same
# state. Positions: the float32 CoG (|c| up to a few m, ulp 2.4e-7 m) and the
# point positions built from it; velocities: the penalty forces turn ~3e-7 m of
# point-position rounding into ~1.5e-3 N per contact point, i.e. ~1e-5 m/s over
# a frame, and the friction correction divides the fitted slip's rounding
# (~1e-9 m) by dt; the torso height is accumulated from float32 values. Each
# bound is a few times the largest deviation measured on the MI355X over the
# parity workloads (about 2e5 robot-frames).
FRAME_TOL = {
    "pos": 2e-6,      # m, CoG
    "ang": 2e-6,      # rad, orientation
    "vel": 1e-4,      # m/s
    "omega": 2e-3,    # rad/s
    "joint": 2e-6,    # rad, joint angles and previous joint angles
    "tele_h": 4e-6,   # m, one frame's torso height
}
# Fragile decisions searched for a frame beyond FRAME_TOL: look-ups and contact
# tests within 1e-5 m (tens of float32 position ulps), the fit's spread test
# within 1e-4 relative, and the static-friction comparison within 1e-2
# relative (a sticking frame's mean slip of ~1e-6 m is a float32 difference of
# displacements ~1e-4 m; only the slipping-frame counter depends on it).
FRAGILE_MARGIN_M = 1e-5
FRAGILE_MARGIN_REL = 1e-4
FRAGILE_MARGIN_CAP = 1e-2
MAX_FLIP_SEARCH = 12   # decisions tried in pairs when no single flip explains a frame
MAX_FLIP_ALL = 6       # up to this many logged decisions, every subset is tried
# conditioning of a frame beyond FRAME_TOL: ENSEMBLE oracle frames from the state
# perturbed by one float32 rounding; the bound grows by SENS x their spread
ENSEMBLE = 8
ENSEMBLE_REL = 2.0 ** -23
SENS = 4.0

# per-test summaries for the terminal report (filled by assert_windows)
REPORT = []


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
    tele = gw.read_state(N.F_TELE)
    for i, st in zip(idx, states):
        J = J_of(i)
        body[:, i] = st[:13].astype(np.float32)
        q[:J, i] = st[O.HDR:O.HDR + J].astype(np.float32)
        qp[:J, i] = st[O.HDR + J:O.HDR + 2 * J].astype(np.float32)
        step[i] = int(st[O.STEP])
        flags[i] = int(st[O.FLAGS])
        tele[:, i] = st[O.TELE:O.TELE + 4]
    gw.write_state(N.F_BODY, body)
    gw.write_state(N.F_JOINT, q)
    gw.write_state(N.F_JOINT_PREV, qp)
    gw.write_state(N.F_STEP, step)
    gw.write_state(N.F_FLAGS, flags)
    gw.write_state(N.F_TELE, tele)


class _Reader:
    """Reads the state rows of a few instances; for large worlds the columns
    are gathered on the device so only the sampled ones cross to the host."""

    FIELDS = (N.F_BODY, N.F_JOINT, N.F_JOINT_PREV, N.F_STEP, N.F_FLAGS, N.F_TELE)

    def __init__(self, gw, idx):
        self.gw = gw
        self.idx = list(idx)
        self.dev = None
        if gw.n_instances >= 1024:
            import torch
            tdt = {np.float32: torch.float32, np.int32: torch.int32, np.float64: torch.float64}
            self.dev = {}
            for f in self.FIELDS:
                shape, dt = gw._field_shape(f)
                self.dev[f] = torch.empty(shape, dtype=tdt[dt], device="cuda")
            self.col = torch.as_tensor(self.idx, dtype=torch.long, device="cuda")

    def read(self):
        """{field: array whose last axis runs over idx}."""
        if self.dev is None:
            return {f: self.gw.read_state(f)[..., self.idx] for f in self.FIELDS}
        out = {}
        for f in self.FIELDS:
            t = self.gw.read_state(f, out=self.dev[f])
            out[f] = t.index_select(t.dim() - 1, self.col).cpu().numpy()
        return out


def states_from(rows, J_of, idx):
    """Oracle-layout float64 state vectors of idx from the rows _Reader.read gave."""
    out = []
    for k, i in enumerate(idx):
        J = J_of(i)
        st = np.zeros(O.HDR + 2 * J)
        st[:13] = rows[N.F_BODY][:, k]
        st[O.STEP] = rows[N.F_STEP][k]
        st[O.FLAGS] = rows[N.F_FLAGS][k]
        st[O.TELE:O.TELE + 4] = rows[N.F_TELE][:, k]
        st[O.HDR:O.HDR + J] = rows[N.F_JOINT][:J, k]
        st[O.HDR + J:] = rows[N.F_JOINT_PREV][:J, k]
        out.append(st)
    return out


def read_states(gw, idx, J_of):
    """GPU states of instances idx as oracle-layout float64 vectors."""
    idx = list(idx)
    return states_from(_Reader(gw, idx).read(), J_of, idx)


def quat_angle(q1, q2):
    """Geodesic angle between two unit quaternions."""
    d = abs(float(np.dot(q1, q2)) / (np.linalg.norm(q1) * np.linalg.norm(q2)))
    return 2.0 * math.acos(min(1.0, d))


def frame_errors(h, g, J):
    """Per-group deviations of GPU state g from oracle state h (same layout)."""
    jq = slice(O.HDR, O.HDR + 2 * J)
    return {
        "pos": float(np.abs(h[0:3] - g[0:3]).max()),
        "ang": quat_angle(h[3:7], g[3:7]),
        "vel": float(np.abs(h[7:10] - g[7:10]).max()),
        "omega": float(np.abs(h[10:13] - g[10:13]).max()),
        "joint": float(np.abs(h[jq] - g[jq]).max()) if J else 0.0,
        "tele_h": abs(float(h[O.TELE] - g[O.TELE])),
        "tele_n": max(abs(float(h[O.TELE + 1] - g[O.TELE + 1])),
                      abs(float(h[O.TELE + 2] - g[O.TELE + 2]))),
        "int": float(int(h[O.STEP]) != int(g[O.STEP]) or int(h[O.FLAGS]) != int(g[O.FLAGS])),
    }


def frame_within(e, tol=FRAME_TOL):
    return (all(e[k] <= tol[k] for k in tol) and e["tele_n"] == 0.0 and e["int"] == 0.0)


def describe(dec):
    s, k, kind = dec[:3]
    where = f"point {k}" if k >= 0 else "robot"
    return f"{O.STAGE_NAMES[s]}, {where}, {O.KIND_NAMES[kind]}"


def frame_spread(ow, i, before, ref, seed):
    """Largest deviation, per quantity, of ENSEMBLE oracle frames taken from
    inputs perturbed by one float32 rounding from the oracle frame `ref` of the
    unperturbed ones: every component of the body state and joint angles
    (relative ENSEMBLE_REL, uniform), and every controller parameter by one
    float32 ulp up or down (the joint angles a frame commands are float32
    numbers too)."""
    J = ow.morph_of(i).n_joints
    rng = np.random.default_rng(seed)
    out = {k: 0.0 for k in FRAME_TOL}
    ctrl = ow.ctrl[i]
    c0 = ctrl.copy()
    try:
        for _ in range(ENSEMBLE):
            up = rng.random(c0.shape) < 0.5
            ctrl[...] = np.where(up, np.nextafter(c0, np.float32(np.inf)),
                                 np.nextafter(c0, np.float32(-np.inf)))
            p = before.copy()
            for a, b in ((0, 13), (O.HDR, O.HDR + 2 * J)):
                p[a:b] *= 1.0 + rng.uniform(-1.0, 1.0, b - a) * ENSEMBLE_REL
            ow.step(i, p)
            e = frame_errors(ref, p, J)
            for k in out:
                out[k] = max(out[k], e[k])
    finally:
        ctrl[...] = c0
    return out


def check_frame(ow, i, before, got, tol=FRAME_TOL):
    """One GPU frame of instance i (state `before` -> `got`) against the oracle
    frame from `before`. Returns (verdict, errors, info): verdict "ok", "cond"
    (within the bound widened by the frame's own float32 sensitivity; info: the
    widened bound), "flip" (info: the decisions flipped, with their distances)
    or "fail" (info: the frame's fragile decisions)."""
    J = ow.morph_of(i).n_joints
    h = before.copy()
    log = ow.step_ex(i, h, FRAGILE_MARGIN_M, FRAGILE_MARGIN_REL, margin_cap=FRAGILE_MARGIN_CAP)
    e = frame_errors(h, got, J)
    if frame_within(e, tol):
        return "ok", e, None
    spread = frame_spread(ow, i, before, h, seed=int(before[O.STEP]) * 7919 + i)
    wide = {k: tol[k] + SENS * spread[k] for k in tol}
    if frame_within(e, wide):
        return "cond", e, wide
    seen, cands = set(), []
    for dec in sorted(log, key=lambda d: d[3]):
        if dec[:3] not in seen:
            seen.add(dec[:3])
            cands.append(dec)
    if len(cands) <= MAX_FLIP_ALL:
        # few decisions: every subset (a point near a cell corner may take its
        # x and y look-ups at P^n, at P* and under the torso all the other way)
        trials = [list(p) for k in range(1, len(cands) + 1)
                  for p in itertools.combinations(cands, k)]
    else:
        trials = [[c] for c in cands]
        trials += [list(p) for p in itertools.combinations(cands[:MAX_FLIP_SEARCH], 2)]
    for flips in trials:
        h = before.copy()
        ow.step_ex(i, h, FRAGILE_MARGIN_M, FRAGILE_MARGIN_REL, flips=[d[:3] for d in flips],
                   margin_cap=FRAGILE_MARGIN_CAP)
        e2 = frame_errors(h, got, J)
        if frame_within(e2, wide):
            return "flip", e2, flips
    return "fail", e, cands


class WindowStats:
    def __init__(self, start, inst, start_state=None, length=0):
        self.start_frame = start
        self.inst = inst
        self.start_state = start_state  # the window's (float32-rounded) start state
        self.length = length
        self.storage = None     # the float32-storage oracle's window deviation, when computed
        self.cog = self.pts = self.joint = self.orient = 0.0
        self.frames = 0
        self.flips = []         # (frame, decisions) of frames explained by a flip
        self.cond = []          # (frame, errors) of ill-conditioned frames within the widened bound
        self.failed = []        # (frame, errors, fragile decisions) of unexplained frames
        self.frame_max = {}     # largest one-frame deviations of the frames within FRAME_TOL

    def update(self, ref, got, Pref, Pgot, J):
        self.cog = max(self.cog, float(np.abs(ref[:3] - got[:3]).max()))
        self.orient = max(self.orient, quat_angle(ref[3:7], got[3:7]))
        if J:
            self.joint = max(self.joint, float(np.abs(ref[O.HDR:O.HDR + J]
                                                      - got[O.HDR:O.HDR + J]).max()))
        if Pref is not None:
            self.pts = max(self.pts, float(np.abs(Pref - Pgot).max()))

    def note_frame(self, frame, verdict, e, info):
        self.frames += 1
        if verdict == "ok":
            for k in FRAME_TOL:
                self.frame_max[k] = max(self.frame_max.get(k, 0.0), e[k])
        elif verdict == "cond":
            self.cond.append((frame, e))
        elif verdict == "flip":
            self.flips.append((frame, info))
        else:
            self.failed.append((frame, e, info))

    def ok(self):
        return (self.cog <= POS_TOL and self.pts <= POS_TOL and self.joint <= ANG_TOL
                and self.orient <= ANG_TOL)

    def verified(self):
        return not self.failed

    def __repr__(self):
        return (f"cog {self.cog:.2e} m, points {self.pts:.2e} m, joints {self.joint:.2e} rad, "
                f"orientation {self.orient:.2e} rad")


def run_windows(ow, gw, idx, starts, length=200, check_points=True, tol=FRAME_TOL):
    """For each window start s: the oracle trajectory at frame s, rounded to FP32,
    is written to the GPU; both advance `length` frames one at a time and are
    compared every frame (window check), and every GPU frame is checked against
    the oracle frame from the GPU's own previous state (frame check). At the end
    of each window the GPU's own point positions are compared with the oracle's
    positions of the GPU state. Returns one WindowStats per (start, instance)."""
    idx = list(idx)
    J_of = lambda i: ow.morph_of(i).n_joints
    reader = _Reader(gw, idx)
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
        stats = {i: WindowStats(s, i, start[i].copy(), length) for i in idx}
        before = states_from(reader.read(), J_of, idx)
        for k in range(length):
            gw.step_n(1)
            got = states_from(reader.read(), J_of, idx)
            for n_, i in enumerate(idx):
                ow.step(i, refs[i])
                Pref = ow.points(i, refs[i]) if check_points else None
                Pgot = ow.points(i, got[n_]) if check_points else None
                stats[i].update(refs[i], got[n_], Pref, Pgot, J_of(i))
                verdict, e, info = check_frame(ow, i, before[n_], got[n_], tol)
                stats[i].note_frame(s + k, verdict, e, info)
            before = got
        if check_points:
            P = gw.read_points()
            for n_, i in enumerate(idx):
                n_pts = ow.morph_of(i).n_points
                own = ow.points(i, before[n_])
                dev = float(np.abs(P[i, :n_pts] - own).max())
                # the GPU's own float32 point positions of its state
                assert dev <= 4 * FRAME_TOL["pos"], (s, i, dev)
        results += [stats[i] for i in idx]
    return results


def summarize(label, results):
    """One line per test for the terminal report, and the windows beyond tolerance."""
    n = len(results)
    over = [r for r in results if not r.ok()]
    flips = sum(len(r.flips) for r in results)
    cond = sum(len(r.cond) for r in results)
    frames = sum(r.frames for r in results)
    worst = max(results, key=lambda r: max(r.cog, r.pts) / POS_TOL
                + max(r.joint, r.orient) / ANG_TOL)
    fmax = {}
    for r in results:
        for k, v in r.frame_max.items():
            fmax[k] = max(fmax.get(k, 0.0), v)
    line = (f"{label}: {n} windows, {len(over)} beyond 1e-4 m / 1e-3 rad (verified frame by "
            f"frame), {frames} frames checked, {flips} with a flipped fragile decision, {cond} "
            f"ill-conditioned within the widened bound; worst "
            f"window (start {worst.start_frame}, inst {worst.inst}): {worst}; largest one-frame "
            f"deviation " + ", ".join(f"{k} {v:.1e}" for k, v in fmax.items()))
    REPORT.append(line)
    return line, over


def storage_window(ow, r):
    """The window of r run twice by the oracle from its start state: in float64,
    and with the state rounded to float32 after every frame (float32 storage of
    the state and nothing else). Returns the deviation between the two runs, as
    a WindowStats measured like the GPU's window."""
    i, J = r.inst, ow.morph_of(r.inst).n_joints
    a, b = r.start_state.copy(), r.start_state.copy()
    out = WindowStats(r.start_frame, i)
    for _ in range(r.length):
        ow.step(i, a)
        ow.step(i, b)
        b = round_state(b)
        out.update(a, b, ow.points(i, a), ow.points(i, b), J)
    return out


def assert_windows(results, label, say=print, ow=None):
    """Every frame verified; every window within tolerance, or beyond it with
    every frame verified. A window beyond tolerance whose start, run by the
    oracle with only its state rounded to float32 after each frame, also leaves
    the tolerance is limited by float32 storage of the state (chaotic contact
    amplifies that rounding alone past 1e-4 m within the window); at most
    MAX_ATTRIBUTED_FRACTION of the windows may be beyond tolerance without that
    explanation."""
    line, over = summarize(label, results)
    say(line)
    for r in results:
        for frame, decs in r.flips:
            say(f"  frame {frame} inst {r.inst}: flipped "
                + "; ".join(f"{describe(d)} at {d[3]:.1e}" for d in decs))
    for r in over:
        if ow is not None and r.start_state is not None and r.length:
            r.storage = storage_window(ow, r)
        lim = r.storage is not None and not r.storage.ok()
        say(f"  beyond tolerance, every frame verified: start {r.start_frame} inst {r.inst}: {r}"
            + (f"; float32 storage alone: {r.storage}" if r.storage is not None else ""))
    unexplained = [r for r in over if r.storage is None or r.storage.ok()]
    if ow is not None and over:
        note = (f"{label}: of {len(over)} windows beyond tolerance, {len(over) - len(unexplained)} "
                f"leave it under float32 storage of the state alone")
        say(note)
        REPORT.append(note)
    bad = [r for r in results if not r.verified()]
    for r in bad:
        for frame, e, cands in r.failed[:3]:
            say(f"  FAIL frame {frame} inst {r.inst}: "
                + ", ".join(f"{k} {v:.2e}" for k, v in e.items())
                + f"; fragile decisions tried: {len(cands)}")
    assert not bad, f"{label}: {len(bad)} windows with frames that match no oracle frame"
    assert len(unexplained) <= MAX_ATTRIBUTED_FRACTION * len(results), \
        f"{label}: {len(unexplained)} of {len(results)} windows beyond tolerance, not explained " \
        f"by float32 storage of the state"
