"""Seeded synthetic inputs for the legged-robot step.

This module is shared by the FP64 oracle and the HIP path, and it holds none of
the step's arithmetic: it only lays out geometry, terrain and controller
parameters as plain arrays. Both sides read the same float32 arrays.

Table format of one robot (a "morphology"), in the construction frame (the
torso frame at the zero pose, z up, SI units):

* ``points``  float32 [N, 4]  -- x, y, z, mass of every mass point (Sec. III-A:
  the robot is a set of mass points; a body's mass is spread evenly over its
  points).
* ``pt_link`` int32 [N]       -- rigid link that owns each point (0 = torso).
* ``parent``  int32 [L]       -- parent link of each link, ``parent[0] == -1``,
  ``parent[l] < l``.
* ``joint``   float32 [L, 8]  -- hinge of link l (Sec. IV-B, createJoint): the
  anchor point (3) and unit axis (3) in the construction frame, then the lower
  and upper joint limits in rad. Row 0 (torso) is unused. Joint ``j`` drives
  link ``j + 1``.

A controller is float32 [J, 3] = (A, f, phi) per joint: the commanded angle is
A sin(2 pi f t + phi) about the zero pose.

A heightfield is a piecewise-constant look-up table (Sec. III-A) with ``nx`` by
``ny`` cells of side ``1/s`` metres whose corner cell starts at (x0, y0).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NO_LIMIT = 1.0e30  # joint limit value meaning "unlimited"


@dataclass
class Morph:
    points: np.ndarray   # float32 [N, 4]
    pt_link: np.ndarray  # int32 [N]
    parent: np.ndarray   # int32 [L]
    joint: np.ndarray    # float32 [L, 8]
    name: str = ""

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_links(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_joints(self) -> int:
        return self.n_links - 1


@dataclass
class Heightfield:
    nx: int
    ny: int
    s: float          # cells per metre (the paper's scaling factor)
    x0: float
    y0: float
    H: np.ndarray     # float32 [ny, nx]
    height_fn: object = None   # analytic height used to place robots (may be None)

    def ground(self, x: float, y: float) -> float:
        """Height of the analytic terrain the table was sampled from."""
        if self.height_fn is None:
            return 0.0
        return float(self.height_fn(x, y))


@dataclass
class Params:
    dt: float = 1.0e-3
    K: int = 1                  # joint-update interval in steps
    g: tuple = (0.0, 0.0, -9.81)
    mu: float = 1.0             # friction coefficient; math.inf = always stick
    k_n: float = 5000.0         # normal penalty stiffness per point, N/m
    zeta: float = 5.0           # Hunt-Crossley damping, s/m
    eps: float = 1.0e-4         # LSQ spread threshold, m
    friction_weighting: bool = False  # friction fit weighted by each point's normal force
    hf_bilinear: bool = False   # height map read bilinearly between cell centres
    max_joint_rate: float = 0.0  # rad/s a joint may turn (0: no limit)
    friction_6dof: bool = False  # friction fit over the full rigid motion in 3-D


@dataclass
class Workload:
    """A batch: morphologies, instance -> morphology map, controllers, start poses."""
    params: Params
    hf: Heightfield
    morphs: list
    inst_morph: np.ndarray     # int32 [I]
    ctrl: list                 # per instance float32 [J_i, 3]
    pose: np.ndarray           # float32 [I, 7]: torso-origin position (3), quaternion w,x,y,z
    n_steps: int = 1000
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_instances(self) -> int:
        return int(self.inst_morph.shape[0])


# ----------------------------------------------------------------------------
# geometry helpers (point placement only)
# ----------------------------------------------------------------------------

def _cross(a, b):
    """Cross product of two 3-vectors (the component formulas, as numpy's)."""
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def _ring(center, direction, radius, n):
    """n points on a circle of given radius around `center`, normal `direction`."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    helper = np.array([0.0, 0.0, 1.0]) if abs(d[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = _cross(d, helper)
    e1 /= np.linalg.norm(e1)
    e2 = _cross(d, e1)
    ang = 2.0 * np.pi * np.arange(n) / n
    return (np.asarray(center, dtype=np.float64)[None, :]
            + radius * (np.cos(ang)[:, None] * e1[None, :] + np.sin(ang)[:, None] * e2[None, :]))


def _cylinder_cloud(p0, p1, radius, n):
    """Point cloud of a thin cylinder: two rings at its end caps (n points total)."""
    n0 = (n + 1) // 2
    n1 = n - n0
    d = np.asarray(p1, dtype=np.float64) - np.asarray(p0, dtype=np.float64)
    return np.concatenate([_ring(p0, d, radius, n0), _ring(p1, d, radius, n1)], axis=0)


def _torso_cloud(lx=0.30, ly=0.20, lz=0.05, gx=8, gy=4):
    """Box torso: top and bottom faces each carry a gx-by-gy grid spanning the face."""
    xs = np.linspace(-lx / 2, lx / 2, gx)
    ys = np.linspace(-ly / 2, ly / 2, gy)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pts = []
    for z in (-lz / 2, lz / 2):
        pts.append(np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1))
    return np.concatenate(pts, axis=0)


class _Builder:
    def __init__(self):
        self.pts, self.m, self.link = [], [], []
        self.parent = [-1]
        self.joint = [np.zeros(8)]

    def add_points(self, xyz, mass_total, link):
        xyz = np.asarray(xyz, dtype=np.float64)
        self.pts.append(xyz)
        self.m.append(np.full(len(xyz), mass_total / len(xyz)))
        self.link.append(np.full(len(xyz), link, dtype=np.int32))

    def add_link(self, parent, anchor, axis, lo=-NO_LIMIT, hi=NO_LIMIT):
        axis = np.asarray(axis, dtype=np.float64)
        axis = axis / np.linalg.norm(axis)
        self.parent.append(parent)
        self.joint.append(np.concatenate([np.asarray(anchor, dtype=np.float64), axis, [lo, hi]]))
        return len(self.parent) - 1

    def build(self, name):
        xyz = np.concatenate(self.pts, axis=0)
        m = np.concatenate(self.m)
        pts = np.concatenate([xyz, m[:, None]], axis=1).astype(np.float32)
        return Morph(points=pts, pt_link=np.concatenate(self.link).astype(np.int32),
                     parent=np.asarray(self.parent, dtype=np.int32),
                     joint=np.asarray(self.joint, dtype=np.float64).astype(np.float32), name=name)


def legged(leg_x, link_len, link_mass, pts_per_link, torso_mass=2.0, hip_y=0.10,
           ring_radius=0.01, name="legged"):
    """A torso with legs on both sides.

    ``leg_x``: hip x positions (one leg per side at each); ``link_len``/``link_mass``/
    ``pts_per_link``: per leg, a list over that leg's links. The first joint of a
    leg yaws about the torso z axis; the others pitch about (outward x z), so a
    positive angle raises the foot. At the zero pose every link points outward,
    horizontal, except the last, which points straight down.
    """
    b = _Builder()
    b.add_points(_torso_cloud(), torso_mass, 0)
    leg = 0
    for side in (+1.0, -1.0):
        out = np.array([0.0, side, 0.0])
        pitch = np.cross(out, [0.0, 0.0, 1.0])
        for hx in leg_x:
            lens, masses, npts = link_len[leg], link_mass[leg], pts_per_link[leg]
            leg += 1
            p = np.array([hx, side * hip_y, 0.0])
            parent = 0
            nl = len(lens)
            for k in range(nl):
                axis = [0.0, 0.0, 1.0] if k == 0 else pitch
                d = np.array([0.0, 0.0, -1.0]) if (k == nl - 1 and nl > 1) else out
                q = p + lens[k] * d
                lid = b.add_link(parent, p, axis)
                b.add_points(_cylinder_cloud(p, q, ring_radius, npts[k]), masses[k], lid)
                parent, p = lid, q
    return b.build(name)


def hexapod() -> Morph:
    """The 18-DOF hexapod: torso 0.30x0.20x0.05 m, 2.0 kg, 64 points; six legs of
    coxa 0.05 m/0.1 kg, femur 0.10 m/0.15 kg, tibia 0.12 m/0.1 kg, 16 points per link."""
    legs = 6
    return legged(leg_x=[0.12, 0.0, -0.12],
                  link_len=[[0.05, 0.10, 0.12]] * legs,
                  link_mass=[[0.10, 0.15, 0.10]] * legs,
                  pts_per_link=[[16, 16, 16]] * legs, name="hexapod18")


def random_legged(rng: np.random.Generator) -> Morph:
    """Uneven morphology: 4/6/8 legs, 2-4 joints per leg, link lengths U[0.04, 0.15] m,
    masses U[0.05, 0.3] kg, 200-600 points (torso 64, the rest spread over the leg links,
    at least 8 per link)."""
    n_legs = int(rng.choice([4, 6, 8]))
    jpl = int(rng.choice([2, 3, 4]))
    n_links = n_legs * jpl
    n_min = max(200, 64 + 8 * n_links)
    n_tot = int(rng.integers(n_min, 601))
    per = np.full(n_links, (n_tot - 64) // n_links, dtype=np.int64)
    per[: (n_tot - 64) - per.sum()] += 1
    lens = rng.uniform(0.04, 0.15, size=(n_legs, jpl))
    masses = rng.uniform(0.05, 0.30, size=(n_legs, jpl))
    half = n_legs // 2
    leg_x = list(np.linspace(-0.12, 0.12, half)) if half > 1 else [0.0]
    m = legged(leg_x=leg_x, link_len=lens.tolist(), link_mass=masses.tolist(),
               pts_per_link=per.reshape(n_legs, jpl).tolist(),
               name=f"legs{n_legs}x{jpl}_n{n_tot}")
    m.meta_drop = float(lens[:, -1].max())  # longest downward link
    return m


# ----------------------------------------------------------------------------
# terrain
# ----------------------------------------------------------------------------

def sensor_rays(m: Morph) -> tuple:
    """Six range-sensor rays of a legged robot, in its construction frame: from
    the torso's centre (mean of the root link's points) straight down 0.5 m and
    0.5 m down-and-out towards +x, -x, +y, -y at 45 degrees; and from the
    centre of the first leaf link's points straight down 0.3 m.
    Returns (rays [6, 6] float32 start+end, ray_link [6] int32)."""
    pts = m.points[:, :3].astype(np.float64)
    c0 = pts[m.pt_link == 0].mean(axis=0)
    children = np.bincount(m.parent[1:], minlength=m.n_links) if m.n_links > 1 else np.zeros(1)
    leaf = int(np.flatnonzero(children == 0)[0]) if m.n_links > 1 else 0
    cf = pts[m.pt_link == leaf].mean(axis=0)
    h = 0.5 / np.sqrt(2.0)
    dirs = [(0, 0, -0.5), (h, 0, -h), (-h, 0, -h), (0, h, -h), (0, -h, -h)]
    rays = [np.r_[c0, c0 + np.asarray(d)] for d in dirs] + [np.r_[cf, cf + [0, 0, -0.3]]]
    links = [0] * 5 + [leaf]
    return np.asarray(rays, np.float32), np.asarray(links, np.int32)


def random_rays(m: Morph, n: int, rng: np.random.Generator) -> tuple:
    """n rays on random links of m: starts at random points of the link (jittered
    by up to 2 cm), random directions, lengths U[0.05, 1.0] m."""
    link = rng.integers(0, m.n_links, n).astype(np.int32)
    rays = np.zeros((n, 6), np.float32)
    for k in range(n):
        own = np.flatnonzero(m.pt_link == link[k])
        p = m.points[rng.choice(own), :3].astype(np.float64) + rng.uniform(-0.02, 0.02, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        rays[k] = np.r_[p, p + d * rng.uniform(0.05, 1.0)]
    return rays, link


def flat_ground(s: float = 50.0) -> Heightfield:
    """Flat plane z = 0: a single cell, every look-up clamps onto it."""
    return Heightfield(nx=1, ny=1, s=s, x0=float(np.float32(-5.12)), y0=float(np.float32(-5.12)),
                       H=np.zeros((1, 1), dtype=np.float32), height_fn=None)


def octave_terrain(seed: int, nx: int = 512, ny: int = 512, cell: float = 0.02,
                   amplitude: float = 0.03) -> Heightfield:
    """Sum of four octaves of random-phase sinusoids, total amplitude `amplitude`.

    h(x, y) = sum_o A_o * (sin(2 pi x / lam_o + ph_o) + sin(2 pi y / lam_o + ps_o)) / 2
    with A_o proportional to 2^-o (sum A_o = amplitude) and lam_o = 2.56 m * 2^-o,
    sampled in float64 at cell centres and stored as float32.
    """
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x7E11]))
    w = 2.0 ** -np.arange(4)
    A = amplitude * w / w.sum()
    lam = 2.56 * w
    ph = rng.uniform(0.0, 2.0 * np.pi, size=4)
    ps = rng.uniform(0.0, 2.0 * np.pi, size=4)

    def h(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        out = np.zeros(np.broadcast(x, y).shape)
        for o in range(4):
            out = out + A[o] * 0.5 * (np.sin(2 * np.pi * x / lam[o] + ph[o])
                                      + np.sin(2 * np.pi * y / lam[o] + ps[o]))
        return out

    x0 = float(np.float32(-0.5 * nx * cell))   # float32-representable origin
    y0 = float(np.float32(-0.5 * ny * cell))
    xc = x0 + (np.arange(nx) + 0.5) * cell
    yc = y0 + (np.arange(ny) + 0.5) * cell
    H = h(xc[None, :], yc[:, None]).astype(np.float32)
    return Heightfield(nx=nx, ny=ny, s=1.0 / cell, x0=x0, y0=y0, H=H, height_fn=h)


# ----------------------------------------------------------------------------
# controllers and batches
# ----------------------------------------------------------------------------

def sinusoid_controller(rng: np.random.Generator, n_joints: int) -> np.ndarray:
    """Per joint (A, f, phi) with A ~ U[0, 0.5] rad, f ~ U[0.5, 2] Hz, phi ~ U[0, 2 pi)."""
    A = rng.uniform(0.0, 0.5, size=n_joints)
    f = rng.uniform(0.5, 2.0, size=n_joints)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_joints)
    return np.stack([A, f, phi], axis=1).astype(np.float32)


def _level_pose(x, y, z):
    return np.array([x, y, z, 1.0, 0.0, 0.0, 0.0], dtype=np.float32)


def config1(seed: int = 1, n_steps: int = 10_000) -> Workload:
    """One 18-DOF hexapod on the flat plane z = 0, torso origin 0.15 m up, at rest."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    return Workload(params=Params(), hf=flat_ground(), morphs=[hexapod()],
                    inst_morph=np.zeros(1, dtype=np.int32),
                    ctrl=[sinusoid_controller(rng, 18)],
                    pose=_level_pose(0.0, 0.0, 0.15)[None, :], n_steps=n_steps,
                    name="hexapod18_flat_1inst")


def hexapod_batch(n_inst: int, seed: int = 2, n_steps: int = 1000, hf: Heightfield | None = None,
                  spread: float = 2.0, name: str | None = None) -> Workload:
    """`n_inst` hexapods on the octave terrain, starts U[-spread, spread]^2, yaw 0,
    torso origin 0.15 m above the terrain, each with its own controller."""
    hf = hf if hf is not None else octave_terrain(seed)
    streams = np.random.SeedSequence(seed).spawn(n_inst + 1)
    pos_rng = np.random.default_rng(streams[-1])
    xy = pos_rng.uniform(-spread, spread, size=(n_inst, 2))
    ctrl = [sinusoid_controller(np.random.default_rng(streams[i]), 18) for i in range(n_inst)]
    pose = np.stack([_level_pose(x, y, hf.ground(x, y) + 0.15) for x, y in xy])
    return Workload(params=Params(), hf=hf, morphs=[hexapod()],
                    inst_morph=np.zeros(n_inst, dtype=np.int32), ctrl=ctrl, pose=pose,
                    n_steps=n_steps, name=name or f"hexapod18_terrain512_{n_inst}inst")


def config2(seed: int = 2, n_inst: int = 4096, n_steps: int = 1000) -> Workload:
    """4,096 hexapods on a 512x512 heightfield at 2 cm, 1,000 steps."""
    return hexapod_batch(n_inst, seed=seed, n_steps=n_steps)


def config3(seed: int = 3, n_inst: int = 16_384, n_steps: int = 5000) -> Workload:
    """Uneven batch: one random legged morphology per instance on the octave terrain."""
    hf = octave_terrain(seed)
    streams = np.random.SeedSequence(seed).spawn(n_inst + 1)
    pos_rng = np.random.default_rng(streams[-1])
    xy = pos_rng.uniform(-2.0, 2.0, size=(n_inst, 2))
    morphs, ctrl, pose = [], [], []
    for i in range(n_inst):
        r = np.random.default_rng(streams[i])
        m = random_legged(r)
        morphs.append(m)
        ctrl.append(sinusoid_controller(r, m.n_joints))
        clearance = 0.03 + m.meta_drop + 0.01
        pose.append(_level_pose(xy[i, 0], xy[i, 1], hf.ground(xy[i, 0], xy[i, 1]) + clearance))
    return Workload(params=Params(), hf=hf, morphs=morphs,
                    inst_morph=np.arange(n_inst, dtype=np.int32), ctrl=ctrl,
                    pose=np.stack(pose), n_steps=n_steps, name=f"uneven_legged_{n_inst}inst")


def subset(w: Workload, idx) -> Workload:
    """The same workload restricted to instances `idx` (morphologies kept shared)."""
    idx = np.asarray(idx, dtype=np.int64)
    return Workload(params=w.params, hf=w.hf, morphs=w.morphs,
                    inst_morph=w.inst_morph[idx].copy(), ctrl=[w.ctrl[i] for i in idx],
                    pose=w.pose[idx].copy(), n_steps=w.n_steps, name=w.name + "_subset",
                    meta=dict(w.meta))
