"""Pins of the range-sensor oracle (rays of the construction API, Sec. IV,
read against the look-up-table ground of Sec. III-A): closed forms on flat and
stepped ground, the clamped map edge, brute-force sampling on the terrain, and
the ray ends against an independent rotation and against the mass points."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from oracle import oracle as O
from paper_2411_05799_amd import workloads as W


def _params(H, s, x0=0.0, y0=0.0):
    H = np.asarray(H, np.float32)
    hf = W.Heightfield(nx=H.shape[1], ny=H.shape[0], s=s, x0=x0, y0=y0, H=H)
    return O.OracleParams(W.Params(), hf)


def test_flat_ground_closed_form():
    """Level ground at h0: the range is len * (z0 - h0) / (z0 - z1) when the ray
    goes from above to at-or-below, 0 from below, the length otherwise."""
    h0 = 0.125
    p = _params(np.full((40, 30), h0), s=10.0, x0=-1.5, y0=-2.0)
    rng = np.random.default_rng(0)
    for _ in range(300):
        A = rng.uniform([-3, -3, -0.5], [3, 3, 1.0])
        B = A + rng.normal(size=3) * rng.uniform(0.01, 2.0)
        L = float(np.linalg.norm(B - A))
        if A[2] <= h0:
            want = 0.0
        elif B[2] <= h0:
            want = L * (A[2] - h0) / (A[2] - B[2])
        else:
            want = L
        assert abs(p.ray_range(A, B) - want) <= 1e-12 * max(1.0, L)


def test_step_terrain_wall_and_plateau():
    """A 0.1 m step at x = 5 (cells of 0.1 m): a level ray below the step's top
    stops at the wall; a descending ray that clears the wall lands on the
    plateau; one leaving the plateau downhill above both levels misses."""
    H = np.zeros((20, 100), np.float32)
    H[:, 50:] = 0.1
    top = float(np.float32(0.1))            # the stored height
    p = _params(H, s=10.0)
    # level ray at z = 0.05 from x = 4.2 to x = 6.0: hits the wall at x = 5
    assert abs(p.ray_range([4.2, 0.33, 0.05], [6.0, 0.33, 0.05]) - 0.8) < 1e-12
    # z = 0.3 - 0.3 t over x = 4 + 2 t: at the wall (t = 0.5) z = 0.15 > 0.1;
    # it meets the plateau at t = 2/3
    A, B = np.array([4.0, 0.5, 0.3]), np.array([6.0, 0.5, 0.0])
    want = (0.3 - top) / 0.3 * np.linalg.norm(B - A)
    assert abs(p.ray_range(A, B) - want) < 1e-12
    # from the plateau down to z = 0.05 over the low side: above 0.1 while over
    # the plateau (t < 0.5), above 0 after
    A, B = np.array([6.0, 0.5, 0.3]), np.array([4.0, 0.5, 0.05])
    assert abs(p.ray_range(A, B) - np.linalg.norm(B - A)) < 1e-12
    # straight down onto the plateau and onto the low side
    assert abs(p.ray_range([5.55, 1.0, 0.7], [5.55, 1.0, -0.3]) - (0.7 - top)) < 1e-12
    assert abs(p.ray_range([4.55, 1.0, 0.7], [4.55, 1.0, -0.3]) - 0.7) < 1e-12


def test_map_edge_is_clamped():
    """Beyond the map the edge cells' heights continue (clamped indices)."""
    H = np.zeros((10, 10), np.float32)
    H[:, -1] = 0.5                          # last column, x in [0.9, 1.0)
    p = _params(H, s=10.0)
    # wholly past the +x edge at z = 0.4: under the clamped edge height
    assert p.ray_range([1.5, 0.5, 0.4], [2.5, 0.5, 0.4]) == 0.0
    # past the -x edge the clamped first column is 0: z = 0.4 -> 0.2 never reaches it
    L = math.hypot(1.0, 0.2)
    assert abs(p.ray_range([-1.5, 0.5, 0.4], [-2.5, 0.5, 0.2]) - L) < 1e-12
    # coming in from -x at z = 0.4 it meets the high column's face at x = 0.9
    assert abs(p.ray_range([-0.6, 0.5, 0.4], [1.4, 0.5, 0.4]) - 1.5) < 1e-12


def _below(hf, P):
    """Whether points P [n, 3] are at or below the ground, the cell decided as
    the step decides it (float32 (x - x0) * s, floor, clamp)."""
    def idx(x, x0, cnt):
        u = (x.astype(np.float32) - np.float32(x0)) * np.float32(hf.s)
        i = np.floor(u).astype(np.int64)
        return np.clip(np.where(u >= 0, i, 0), 0, cnt - 1)
    i = idx(P[:, 0], hf.x0, hf.nx)
    j = idx(P[:, 1], hf.y0, hf.ny)
    return P[:, 2] <= hf.H[j, i].astype(np.float64)


def test_terrain_against_brute_force_sampling():
    """On the 2 cm octave terrain, with 200,001 samples t_k = k / n per ray: the
    range lies between the last sample above the ground and the first one at
    or below it; when no sample is below, it is the length or the point just
    past it is below (a hit between two samples)."""
    hf = W.octave_terrain(6, nx=128, ny=128)
    p = O.OracleParams(W.Params(), hf)
    rng = np.random.default_rng(1)
    n = 200_000
    t = np.arange(n + 1, dtype=np.float64) / n
    hits = 0
    for _ in range(60):
        A = np.r_[rng.uniform(-1.2, 1.2, 2), rng.uniform(0.0, 0.15)]
        d = rng.normal(size=3)
        d[2] = -abs(d[2]) * rng.uniform(0.05, 1.0)
        B = A + d / np.linalg.norm(d) * rng.uniform(0.1, 1.5)
        L = float(np.linalg.norm(B - A))
        r = p.ray_range(A, B)
        below = np.flatnonzero(_below(hf, A[None, :] + t[:, None] * (B - A)[None, :]))
        if below.size == 0:
            if r < L * (1.0 - 1e-12):       # (a hit at the very end rounds either way)
                after = A + min(1.0, r / L + 1e-9) * (B - A)
                assert _below(hf, after[None, :])[0], (r, L)
        elif below[0] == 0:
            assert r == 0.0
        else:
            k = int(below[0])
            hits += 1
            assert L * t[k - 1] - 1e-12 <= r <= L * t[k] + 1e-12, (r / L, t[k - 1], t[k])
    assert hits >= 20


def test_ray_ends_on_the_root_follow_an_independent_rotation():
    """A box of eight equal corner masses centred on the origin has g_b = 0, so
    a root-link ray end p is at c + R(Q) p (R from scipy's quaternion map)."""
    box = W.Morph(points=np.array([[sx * 0.1, sy * 0.05, sz * 0.025, 0.125]
                                   for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                                  np.float32),
                  pt_link=np.zeros(8, np.int32), parent=np.array([-1], np.int32),
                  joint=np.zeros((1, 8), np.float32), name="box")
    w = W.Workload(params=W.Params(), hf=W.flat_ground(), morphs=[box],
                   inst_morph=np.zeros(1, np.int32), ctrl=[np.zeros((0, 3), np.float32)],
                   pose=np.array([[0, 0, 0.3, 1, 0, 0, 0]], np.float32))
    ow = O.OracleWorld(w)
    rng = np.random.default_rng(2)
    rays, links = W.random_rays(box, 5, rng)
    for _ in range(5):
        st = ow.init_state(0)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        st[O.C_:O.C_ + 3] = rng.uniform(-1, 1, 3)
        st[O.Q_:O.Q_ + 4] = q
        S, E = ow.ray_ends(0, st, rays, links)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        want_S = st[:3] + rays[:, :3].astype(np.float64) @ R.T
        want_E = st[:3] + rays[:, 3:].astype(np.float64) @ R.T
        assert np.abs(S - want_S).max() < 1e-12 and np.abs(E - want_E).max() < 1e-12


def test_ray_ends_coincide_with_mass_points_of_their_link():
    """A ray whose ends sit at two mass points of a hexapod's link ends where the
    step puts those points, at any joint angles and pose."""
    m = W.hexapod()
    w = W.hexapod_batch(1, seed=4)
    ow = O.OracleWorld(w)
    st = ow.init_state(0)
    ow.run(0, st, 150)
    P = ow.points(0, st)
    rng = np.random.default_rng(3)
    for _ in range(6):
        l = int(rng.integers(0, m.n_links))
        a, b = rng.choice(np.flatnonzero(m.pt_link == l), 2, replace=False)
        rays = np.r_[m.points[a, :3], m.points[b, :3]][None, :]
        S, E = ow.ray_ends(0, st, rays, [l])
        assert np.abs(S[0] - P[a]).max() < 1e-12 and np.abs(E[0] - P[b]).max() < 1e-12
