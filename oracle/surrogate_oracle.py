"""FP64 reference of the simulator-side quantities of the learned surrogate:
state rows, network inputs, the rollout update and the quasi-static joint-torque
proxy used by the controller-search fitness.

TEST INFRASTRUCTURE ONLY: the tests use it to check the GPU kernels; the GPU
library never does.

Definitions (the same ones the library documents):
  state row (width 13 + 2 J): c, Q (w x y z), v, omega, q [J], q_prev [J]
  heading frame of a state: psi = heading of the torso x axis on the ground
    plane; vectors turned by -psi about z; orientations left-multiplied by the
    yaw quaternion of -psi, negated if that leaves w < 0 (the sign chosen for
    the state's own orientation is used for its changes too)
  input (width 13 + 12 J + 64):
    0, 0, c_z - h(c_xy), then Q, v, omega in the heading frame | q | (q - q_prev)/dt |
    clamped commands of frames n .. n+9 (frame-major) |
    8 x 8 patch at 0.08 m, centred on the CoG, turned with the heading (torso x
    axis on the ground plane), minus h(c_xy); index 8 a + b, a along the
    heading, b to its left, offsets (a - 3.5) 0.08 and (b - 3.5) 0.08
  target: the state change over 10 frames, body rows in the heading frame of
    the first state
  rollout update at frame n: body rows + the delta turned back from the heading
    frame of the current state, Q normalised, q = command(n+9), q_prev = command(n+8)
  torque proxy: loads m_k g on every point plus an upward share M |g| / n_low on
    the n_low points less than 0.002 m above the height map; tau_j = axis_j .
    sum over points distal to joint j of (P_k - anchor_j) x load_k; the mean of
    |tau_j| over joints.
Height look-ups use the oracle's own cell rule (index decided in float32).
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

HORIZON = 10
PATCH = 8
PATCH_STEP = 0.08
LOW_BAND = 0.002


def quat_mat(Q):
    w, x, y, z = [float(v) for v in Q]
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_mul(a, b):
    aw, av = a[0], np.asarray(a[1:], np.float64)
    bw, bv = b[0], np.asarray(b[1:], np.float64)
    return np.concatenate([[aw * bw - av @ bv], aw * bv + bw * av + np.cross(av, bv)])


class HeadingFrame:
    """The heading frame of a state with orientation Q."""

    def __init__(self, Q):
        R = quat_mat(Q)
        hn = math.hypot(R[0, 0], R[1, 0])
        self.psi = math.atan2(R[1, 0], R[0, 0]) if hn > 1e-6 else 0.0
        c, s = math.cos(self.psi), math.sin(self.psi)
        self.Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
        self.q_minus = np.array([math.cos(-self.psi / 2), 0.0, 0.0, math.sin(-self.psi / 2)])
        self.q_plus = np.array([math.cos(self.psi / 2), 0.0, 0.0, math.sin(self.psi / 2)])
        self.sign = 1.0 if quat_mul(self.q_minus, Q)[0] >= 0 else -1.0

    def to_frame(self, b):
        """13 body entries (c, Q, v, omega or their changes) world -> heading frame."""
        b = np.asarray(b, np.float64)
        out = np.empty(13)
        for k in (0, 7, 10):
            out[k:k + 3] = self.Rz.T @ b[k:k + 3]
        out[3:7] = self.sign * quat_mul(self.q_minus, b[3:7])
        return out

    def from_frame(self, b):
        b = np.asarray(b, np.float64)
        out = np.empty(13)
        for k in (0, 7, 10):
            out[k:k + 3] = self.Rz @ b[k:k + 3]
        out[3:7] = self.sign * quat_mul(self.q_plus, b[3:7])
        return out


def rodrigues(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def link_transforms(morph, q):
    """Per link (R_l, t_l) mapping construction-frame points of link l to their
    place at joint angles q: T_l(x) = T_parent(Rot(a_l, q_l)(x - o_l) + o_l)."""
    L = morph.n_links
    Rs, ts = [np.eye(3)], [np.zeros(3)]
    for l in range(1, L):
        jt = morph.joint[l].astype(np.float64)
        o, a = jt[:3], jt[3:6]
        Rj = rodrigues(a, float(q[l - 1]))
        p = int(morph.parent[l])
        Rs.append(Rs[p] @ Rj)
        ts.append(Rs[p] @ (o - Rj @ o) + ts[p])
    return Rs, ts


def command(morph, ctrl, j, n, dt):
    A, f, phi = [float(v) for v in ctrl[j]]
    t = n * dt
    qh = A * math.sin(2.0 * math.pi * f * t + phi)
    lo, hi = float(morph.joint[j + 1, 6]), float(morph.joint[j + 1, 7])
    return min(max(qh, lo), hi)


def state_row(st, n_joints, J):
    """Oracle state vector -> state row of width 13 + 2 J."""
    row = np.zeros(13 + 2 * J)
    row[:13] = st[:13]
    q = st[O.HDR:O.HDR + n_joints]
    qp = st[O.HDR + n_joints:O.HDR + 2 * n_joints]
    row[13:13 + n_joints] = q
    row[13 + J:13 + J + n_joints] = qp
    return row


def edge_distance(params, x, y):
    """Distance (in cells) of a point from the nearest cell edge of the table."""
    hf = params
    u = (np.float32(x) - np.float32(hf.x0)) * np.float32(hf.s)
    w = (np.float32(y) - np.float32(hf.y0)) * np.float32(hf.s)
    return float(min(abs(u - round(float(u))), abs(w - round(float(w)))))


class SurrogateOracle:
    def __init__(self, workload):
        self.w = workload
        self.ow = O.OracleWorld(workload)
        self.hp = self.ow.params
        self.J = max(1, max(m.n_links for m in workload.morphs) - 1)
        self.dt = float(workload.params.dt)

    def morph(self, i):
        return self.w.morphs[int(self.w.inst_morph[i])]

    def h(self, x, y):
        return self.hp.height(x, y)

    def near_edge(self, x, y, tol=1e-3):
        return edge_distance(self.w.hf, x, y) < tol

    def patch_points(self, row):
        c = row[:3]
        psi = HeadingFrame(row[3:7]).psi
        ch, sh = math.cos(psi), math.sin(psi)
        pts = []
        for a in range(PATCH):
            for b in range(PATCH):
                u = (a - 0.5 * (PATCH - 1)) * PATCH_STEP
                v = (b - 0.5 * (PATCH - 1)) * PATCH_STEP
                pts.append((c[0] + ch * u - sh * v, c[1] + sh * u + ch * v))
        return pts

    def features(self, i, row, frame):
        """Network input of instance i at state row `row`, frame `frame`."""
        J, m, ctrl = self.J, self.morph(i), self.w.ctrl[i]
        Ji = m.n_links - 1
        x = np.zeros(13 + 12 * J + PATCH * PATCH)
        h0 = self.h(row[0], row[1])
        x[2] = row[2] - h0
        x[3:13] = HeadingFrame(row[3:7]).to_frame(row[:13])[3:13]
        x[13:13 + J] = row[13:13 + J]
        x[13 + J:13 + 2 * J] = (row[13:13 + J] - row[13 + J:13 + 2 * J]) / self.dt
        for k in range(HORIZON):
            for j in range(Ji):
                x[13 + 2 * J + k * J + j] = command(m, ctrl, j, frame + k, self.dt)
        base = 13 + 12 * J
        for idx, (px, py) in enumerate(self.patch_points(row)):
            x[base + idx] = self.h(px, py) - h0
        return x

    def delta(self, row0, row1):
        """Training target: row1 - row0, the body entries in the heading frame of row0."""
        d = np.asarray(row1, np.float64) - np.asarray(row0, np.float64)
        d[:13] = HeadingFrame(row0[3:7]).to_frame(d[:13])
        return d

    def advance(self, i, row, dy, frame):
        J, m, ctrl = self.J, self.morph(i), self.w.ctrl[i]
        out = np.array(row, dtype=np.float64)
        out[:13] += HeadingFrame(row[3:7]).from_frame(dy[:13])
        out[3:7] /= np.linalg.norm(out[3:7])
        out[13:] = 0.0
        for j in range(m.n_links - 1):
            out[13 + j] = command(m, ctrl, j, frame + HORIZON - 1, self.dt)
            out[13 + J + j] = command(m, ctrl, j, frame + HORIZON - 2, self.dt)
        return out

    def heights_near(self, x, y, tol=1e-3):
        """Every table height the look-up of (x, y) could return when the
        coordinates move by up to tol cells (neighbouring cells across a near edge)."""
        hf = self.w.hf

        def cands(v, v0, n):
            u = float((np.float32(v) - np.float32(v0)) * np.float32(hf.s))
            r = round(u)
            idx = {r - 1, r} if abs(u - r) < tol else {math.floor(u)}
            return {min(max(k, 0), n - 1) for k in idx}

        return {float(hf.H[j, i]) for i in cands(x, hf.x0, hf.nx) for j in cands(y, hf.y0, hf.ny)}

    def torque(self, i, row):
        """(mean |tau_j|, ambiguous): ambiguous when some point's load decision
        could go either way under float32 rounding (within 1e-5 m of the band
        edge, or near a cell edge whose neighbouring heights disagree on it)."""
        m = self.morph(i)
        L, Ji = m.n_links, m.n_links - 1
        q = row[13:13 + Ji]
        Rs, ts = link_transforms(m, q)
        pts = m.points[:, :3].astype(np.float64)
        mass = m.points[:, 3].astype(np.float64)
        y = np.array([Rs[l] @ p + ts[l] for p, l in zip(pts, m.pt_link)])
        M = mass.sum()
        gb = (mass[:, None] * y).sum(0) / M
        R = quat_mat(row[3:7])
        c = row[:3]
        arms = (y - gb) @ R.T
        P = c + arms
        gap = np.array([P[k, 2] - self.h(P[k, 0], P[k, 1]) for k in range(len(P))])
        low = gap < LOW_BAND
        ambiguous = bool(np.any(np.abs(gap - LOW_BAND) < 1e-5))
        for k in range(len(P)):
            if ambiguous:
                break
            hs = self.heights_near(P[k, 0], P[k, 1])
            if len(hs) > 1 and len({P[k, 2] - h < LOW_BAND for h in hs}) > 1:
                ambiguous = True
        g = np.asarray(self.w.params.g, np.float64)
        n_low = int(low.sum())
        f_up = -M * g[2] / n_low if n_low else 0.0
        loads = mass[:, None] * g[None, :]
        loads[low, 2] += f_up
        # links distal to each link (itself and its descendants)
        children = {l: [] for l in range(L)}
        for l in range(1, L):
            children[int(m.parent[l])].append(l)

        def subtree(l):
            out = [l]
            for ch in children[l]:
                out += subtree(ch)
            return out

        taus = []
        for l in range(1, L):
            sub = set(subtree(l))
            sel = np.array([int(k) in sub for k in m.pt_link])
            o = m.joint[l, :3].astype(np.float64)
            p = int(m.parent[l])
            anchor = c + R @ (Rs[p] @ o + ts[p] - gb)
            a = m.joint[l, 3:6].astype(np.float64)
            axis = R @ (Rs[p] @ (a / np.linalg.norm(a)))
            mom = np.cross(P[sel] - anchor, loads[sel]).sum(0)
            taus.append(abs(float(axis @ mom)))
        return (float(np.mean(taus)) if taus else 0.0), ambiguous
