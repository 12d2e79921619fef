"""GPU FP32 path vs the FP64 oracle, through the C ABI.

Tolerances: 200-frame windows from identical FP32-representable states agree to
1e-4 m (CoG and every mass point) and 1e-3 rad (joint angles, torso
orientation); long-horizon statistics (distance walked, mean torso height) over
10,000 frames agree to 2%. Integer results (frame counters, flags) and
determinism properties are bit-exact.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_05799_amd import native as N
from paper_2411_05799_amd import workloads as W

from _helpers import (STAT_TOL, assert_windows as _assert_windows, check_frame, describe,
                      gpu_available, read_states, round_state as H_round, run_windows,
                      write_states)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_windows(results, label, ow=None):
    """Every GPU frame is the oracle's frame from the same state (to float32
    rounding, or with a logged fragile decision taken the other way), and every
    window is within 1e-4 m / 1e-3 rad, or beyond it with every frame verified
    (at most a tenth of the windows, not counting windows that float32
    storage of the state alone takes beyond the tolerance)."""
    _assert_windows(results, label, say=say, ow=ow)


def test_placement_matches_oracle():
    say("case: placement config1 + hexapod batch 16")
    for w in (W.config1(), W.hexapod_batch(16, seed=5)):
        ow = O.OracleWorld(w)
        with N.World(w) as gw:
            got = read_states(gw, range(w.n_instances), lambda i: 18)
        for i in range(w.n_instances):
            ref = ow.init_state(i)
            assert np.abs(ref[:13] - got[i][:13]).max() < 2e-6
            assert np.abs(ref[O.HDR:] - got[i][O.HDR:]).max() < 2e-6


def test_config1_windows_all_10k():
    """Config 1 (one hexapod, flat plane): every 200-frame window of 10,000 frames."""
    say("case: config1 windows, 50 x 200 frames")
    w = W.config1()
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, [0], starts=list(range(0, 10_000, 200)))
    assert_windows(res, "config1", ow)


def test_config1_long_horizon_statistics():
    """Distance walked and mean torso height over 10,000 frames within 2%."""
    say("case: config1 long horizon 10k")
    w = W.config1()
    ow = O.OracleWorld(w)
    st = ow.init_state(0)
    c0 = st[:2].copy()
    ow.run(0, st, 10_000)
    with N.World(w) as gw:
        g0 = gw.read_state(N.F_COG)[:2, 0].astype(np.float64)
        gw.step_n(10_000)
        g = read_states(gw, [0], lambda i: 18)[0]
    d_ref = float(np.linalg.norm(st[:2] - c0))
    d_gpu = float(np.linalg.norm(g[:2] - g0))
    h_ref = st[O.TELE] / 10_000
    h_gpu = g[O.TELE] / 10_000
    say(f"distance oracle {d_ref:.4f} m gpu {d_gpu:.4f} m; torso height oracle {h_ref:.5f} "
        f"gpu {h_gpu:.5f} m")
    assert int(g[O.STEP]) == 10_000 and int(g[O.FLAGS]) == 0
    assert abs(d_gpu - d_ref) <= STAT_TOL * d_ref
    assert abs(h_gpu - h_ref) <= STAT_TOL * h_ref


def test_config2_long_horizon_statistics():
    """Terrain is chaotic: after 10,000 frames even the oracle and a copy perturbed
    at float32 scale disagree by tens of percent per robot in distance walked, so
    the check is statistical, on 512 sampled robots of the 4,096: mean torso
    height and mean distance walked within 2%, or within 3 standard errors of
    the paired difference when that is wider."""
    say("case: config2 long horizon, 512 sampled x 10k frames")
    w = W.config2(n_steps=10_000)
    rng = np.random.default_rng(8)
    idx = np.sort(rng.choice(w.n_instances, size=512, replace=False))
    ow = O.OracleWorld(W.subset(w, idx))
    states = ow.init_states()
    c0 = np.array([s[:2] for s in states])
    ow.run_batch(states, 10_000)
    with N.World(w) as gw:
        g0 = gw.read_state(N.F_COG)[:2, idx].T.astype(np.float64)
        gw.step_n(10_000)
        cog = gw.read_state(N.F_COG)[:2, idx].T
        tele = gw.read_state(N.F_TELE)[:, idx]
        flags = gw.read_state(N.F_FLAGS)
    assert not flags.any()
    d_ref = np.linalg.norm(np.array([s[:2] for s in states]) - c0, axis=1)
    d_gpu = np.linalg.norm(cog - g0, axis=1)
    h_ref = np.array([s[O.TELE] for s in states]) / 10_000
    h_gpu = tele[0] / 10_000
    for name, r, g in (("distance walked", d_ref, d_gpu), ("torso height", h_ref, h_gpu)):
        diff = abs(g.mean() - r.mean())
        se = np.std(g - r, ddof=1) / np.sqrt(len(r))
        say(f"{name}: oracle mean {r.mean():.5f} gpu mean {g.mean():.5f} "
            f"(diff {diff / r.mean():.2%}, 3 SE = {3 * se / r.mean():.2%})")
        assert diff <= max(STAT_TOL * r.mean(), 3 * se)


def test_config2_full_size_sampled_windows():
    """4,096 hexapods on the 512x512 terrain at the bench's launch shape: 32 sampled
    instances x 5 windows of 200 frames."""
    say("case: config2 4096 instances, 32 sampled x 5 windows")
    w = W.config2()
    ow = O.OracleWorld(w)
    rng = np.random.default_rng(2)
    idx = sorted(rng.choice(w.n_instances, size=32, replace=False).tolist())
    with N.World(w) as gw:
        from bench import pick_launch
        pick_launch(gw, w)
        res = run_windows(ow, gw, idx, starts=[0, 200, 400, 600, 800])
    assert_windows(res, "config2", ow)


@pytest.mark.parametrize("lanes", [64, 32, 16])
def test_launch_shapes_ragged_batch(lanes):
    """37 hexapods on terrain (a ragged tail for every instances-per-wave) under each
    lanes-per-robot shape, grid and persistent."""
    say(f"case: ragged batch 37, lanes {lanes}")
    w = W.hexapod_batch(37, seed=9, spread=1.0)
    ow = O.OracleWorld(w)
    for persistent in (0, 1):
        with N.World(w) as gw:
            gw.set_launch(lanes_per_instance=lanes, persistent=persistent, waves_per_cu=2)
            res = run_windows(ow, gw, [0, 17, 36], starts=[0, 300])
        assert_windows(res, f"lanes {lanes} persistent {persistent}", ow)


def test_uneven_morphologies():
    """Config-3 style uneven batch (4/6/8 legs, 2-4 joints, 200-600 points)."""
    say("case: uneven batch 48")
    w = W.config3(n_inst=48)
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, list(range(0, 48, 5)), starts=[0, 400])
    assert_windows(res, "uneven", ow)


_C3 = {}


def config3_world():
    """Config 3: 16,384 random legged robots (4/6/8 legs of 2-4 joints, 200-600
    points) on the octave terrain; generated once for the module."""
    if "w" not in _C3:
        _C3["w"] = W.config3(n_inst=16_384, n_steps=10_000)
    return _C3["w"]


def test_config3_full_size_sampled_windows():
    """The 16,384-robot uneven batch in one world at the launch shape the
    autotuner picks for it (the bench's: lanes per robot, links per lane,
    persistent task queue, hipGraph chunks): 32 sampled robots x 5 windows of
    200 frames against the oracle."""
    say("case: config3 16384 uneven robots, 32 sampled x 5 windows")
    w = config3_world()
    ow = O.OracleWorld(w)
    rng = np.random.default_rng(3)
    idx = sorted(rng.choice(w.n_instances, size=32, replace=False).tolist())
    with N.World(w) as gw:
        from bench import pick_launch
        pick_launch(gw, w)
        say(f"launch: {gw.get_launch().as_dict()}")
        res = run_windows(ow, gw, idx, starts=[0, 200, 400, 600, 800])
    assert_windows(res, "config3", ow)


def _state_at(gw, idx, frames, J_of):
    """GPU states of instances idx (float64 oracle layout) at the given frame
    counts, stepping the world forward from its current frame 0."""
    out, at = {}, 0
    for f in sorted(set(frames)):
        gw.step_n(f - at)
        at = f
        got = read_states(gw, idx, J_of)
        for i, st, ff in zip(idx, got, frames):
            if ff == f:
                out[i] = st
    return out


def _gpu_paths(w, launch, windows, J_of):
    """GPU states of instances over frame windows {i: (first, last)}, one
    frame at a time from the world's frame 0 under the given launch."""
    idx = sorted(windows)
    f0 = min(a for a, _ in windows.values())
    f1 = max(b for _, b in windows.values())
    paths = {i: [] for i in idx}
    with N.World(w) as gw:
        gw.set_launch(**launch)
        gw.step_n(f0)
        for f in range(f0, f1 + 1):
            if f > f0:
                gw.step_n(1)
            got = read_states(gw, idx, J_of)
            for i, st in zip(idx, got):
                a, b = windows[i]
                if a <= f <= b:
                    paths[i].append(st)
    return paths


def _assert_path_verified(ow, i, path, what):
    """Every frame of a recorded GPU path of instance i passes the frame judge."""
    counts = {"ok": 0, "cond": 0, "flip": 0, "fail": 0}
    for before, got in zip(path[:-1], path[1:]):
        if int(before[O.FLAGS]) != 0:
            break
        v, e, info = check_frame(ow, i, before, got)
        counts[v] += 1
        assert v != "fail", (i, int(before[O.STEP]), e, [describe(d) for d in info])
    say(f"    {what}, frames {int(path[0][O.STEP])}..{int(path[-1][O.STEP])}: verified frame by "
        f"frame {counts}")
    assert sum(counts.values()) >= len(path) // 2, (i, counts)


def test_config3_long_horizon_statistics_and_flags():
    """10,000 frames of the 16,384-robot uneven batch at the autotuned launch,
    512 robots sampled. Statistics: mean distance walked and mean torso height
    of the robots neither side flags within 2% of the oracle's (or 3 standard
    errors of the paired difference when that is wider: per robot, contact on
    the terrain is chaotic over 10 s). Health flags: some random morphologies
    run away under the method (spin or speed past the limits) on one float32
    or float64 realization of their trajectory and not on the other, so the
    flag rates must agree (within 3 standard errors of the paired difference),
    and every robot flagged by one side only either runs away on the other
    side too when started from the first side's state 50 frames before its
    flag (within 150 frames), or has the GPU frames of that stretch verified
    one by one against the oracle frame from the GPU's own state: a run-away
    built over tens of frames from differences of 1e-8 need not recur on the
    other realization, but no frame on the way to it may be wrong."""
    say("case: config3 long horizon, 512 sampled x 10k frames, health flags")
    n = 10_000
    w = config3_world()
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(w.n_instances, size=512, replace=False))
    J_of = lambda i: w.morphs[int(w.inst_morph[i])].n_joints
    with N.World(w) as gw:
        from bench import pick_launch
        pick_launch(gw, w)          # tunes on scratch copies: the state is untouched
        launch = gw.get_launch().as_dict()
        g_c0 = gw.read_state(N.F_COG)[:2].astype(np.float64)
        gw.step_n(n)
        cog = gw.read_state(N.F_COG)[:2]
        tele = gw.read_state(N.F_TELE)
        gflags = gw.read_state(N.F_FLAGS)
        gstep = gw.read_state(N.F_STEP)
    say(f"launch {launch}; GPU flagged {int((gflags != 0).sum())} of {w.n_instances} robots")
    ow = O.OracleWorld(w)
    states = [ow.init_state(int(i)) for i in idx]
    c0 = np.array([s[:2] for s in states])
    ow.run_batch(states, n, idx=idx)
    of = np.array([int(s[O.FLAGS]) != 0 for s in states])
    gf = gflags[idx] != 0
    diff = gf.astype(float) - of.astype(float)
    se = max(np.std(diff, ddof=1) / np.sqrt(len(idx)), 1.0 / len(idx))
    say(f"flagged among {len(idx)} sampled: GPU {int(gf.sum())}, oracle {int(of.sum())}, both "
        f"{int((gf & of).sum())}")
    assert abs(diff.mean()) <= 3 * se, (gf.sum(), of.sum())
    # one-sided flags: the other side, started from this side's state 50 frames
    # before the flag, runs away too within 150 frames; where it does not, the
    # path that ran away (or, for an oracle-only flag, the GPU's own path from
    # the oracle's state) is verified frame by frame against the oracle frame
    # from the GPU's own state, so no frame of it is wrong.
    gpu_only = [int(i) for i, a, b in zip(idx, gf, of) if a and not b]
    orc_only = [int(i) for i, a, b in zip(idx, gf, of) if b and not a]
    unconfirmed = {}
    if gpu_only:
        back = {i: max(0, int(gstep[i]) - 50) for i in gpu_only}
        with N.World(w) as gw:
            gw.set_launch(**launch)     # the same trajectories, bit for bit
            snap = _state_at(gw, gpu_only, [back[i] for i in gpu_only], J_of)
        for i in gpu_only:
            st = snap[i].copy()
            ow.run(i, st, 150)
            say(f"  robot {i}: GPU flag at frame {int(gstep[i])}; oracle from the GPU state at "
                f"frame {back[i]}: flags {int(st[O.FLAGS])} at frame {int(st[O.STEP])}")
            if int(st[O.FLAGS]) == 0:
                unconfirmed[i] = (back[i], int(gstep[i]))
        if unconfirmed:
            for i, path in _gpu_paths(w, launch, unconfirmed, J_of).items():
                _assert_path_verified(ow, i, path, "GPU path to its flag")
    for i in orc_only:
        k = int(np.nonzero(idx == i)[0][0])
        st = ow.init_state(i)
        ow.run(i, st, max(0, int(states[k][O.STEP]) - 50))
        sub = W.subset(w, [i])
        path = [H_round(st)]
        with N.World(sub) as g1:
            write_states(g1, [0], [path[0]], lambda _: J_of(i))
            for _ in range(150):
                g1.step_n(1)
                path.append(read_states(g1, [0], lambda _: J_of(i))[0])
        f1, s1 = int(path[-1][O.FLAGS]), int(path[-1][O.STEP])
        say(f"  robot {i}: oracle flag at frame {int(states[k][O.STEP])}; GPU from the oracle "
            f"state 50 frames before: flags {f1} at frame {s1}")
        if f1 == 0:
            _assert_path_verified(ow, i, path, "GPU path from the oracle's state")
    ok = ~gf & ~of
    d_ref = np.linalg.norm(np.array([s[:2] for s in states]) - c0, axis=1)[ok]
    d_gpu = np.linalg.norm(cog[:, idx].T - g_c0[:, idx].T, axis=1)[ok]
    h_ref = np.array([s[O.TELE] for s in states])[ok] / n
    h_gpu = tele[0, idx][ok] / n
    for name, r, g in (("distance walked", d_ref, d_gpu), ("torso height", h_ref, h_gpu)):
        dm = abs(g.mean() - r.mean())
        se = np.std(g - r, ddof=1) / np.sqrt(len(r))
        say(f"{name}: oracle mean {r.mean():.5f} gpu mean {g.mean():.5f} "
            f"(diff {dm / abs(r.mean()):.2%}, 3 SE = {3 * se / abs(r.mean()):.2%}) over {len(r)} robots")
        assert dm <= max(STAT_TOL * abs(r.mean()), 3 * se)


def max_robot():
    """1,024 points on 64 links: eight legs, seven of 8 links and one of 7."""
    counts = [8] * 7 + [7]
    per = np.full(63, 960 // 63)
    per[: 960 - per.sum()] += 1
    it = iter(per.tolist())
    m = W.legged(leg_x=list(np.linspace(-0.12, 0.12, 4)),
                 link_len=[[0.05] * (n - 1) + [0.1] for n in counts],
                 link_mass=[[0.05] * n for n in counts],
                 pts_per_link=[[next(it) for _ in range(n)] for n in counts], name="max")
    assert m.n_points == 1024 and m.n_links == 64
    return m


def test_max_size_robot():
    """The largest robot the kernels take: 1,024 points on 64 links."""
    say("case: max-size robot 1024 points 64 links")
    rng = np.random.default_rng(1)
    m = max_robot()
    ctrl = [W.sinusoid_controller(rng, m.n_joints) * np.array([0.3, 1, 1], np.float32)]
    w = W.Workload(params=W.Params(), hf=W.octave_terrain(4), morphs=[m],
                   inst_morph=np.zeros(1, np.int32), ctrl=ctrl,
                   pose=np.array([[0, 0, 0.3, 1, 0, 0, 0]], np.float32))
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, [0], starts=[0, 200, 600])
    assert_windows(res, "max robot", ow)


def test_degenerate_bodies_and_paper_mode():
    """A single mass point (singular inertia), a box in free flight, mu = inf, and the
    paper's own operating point (10 ms frames, joints every 8 frames, 0.1 m cells)."""
    say("case: degenerate bodies / paper mode")
    pt = W.Morph(points=np.array([[0, 0, 0, 1.0]], np.float32), pt_link=np.zeros(1, np.int32),
                 parent=np.array([-1], np.int32), joint=np.zeros((1, 8), np.float32), name="pt")
    box = W.Morph(points=np.array([[sx * 0.1, sy * 0.05, sz * 0.025, 0.125]
                                   for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                                  np.float32),
                  pt_link=np.zeros(8, np.int32), parent=np.array([-1], np.int32),
                  joint=np.zeros((1, 8), np.float32), name="box")
    hexa = W.hexapod()
    cases = [
        (W.Params(), pt, [0.0, 0.0, 0.05]),
        (W.Params(mu=math.inf), box, [0.0, 0.0, 0.06]),
        (W.Params(), box, [0.0, 0.0, 5.0]),
        (W.Params(dt=1e-2, K=8, k_n=1000.0, zeta=5.0), hexa, [0.0, 0.0, 0.15]),
    ]
    for p, m, xyz in cases:
        hf = W.flat_ground(s=10.0) if p.dt > 5e-3 else W.octave_terrain(6)
        rng = np.random.default_rng(3)
        w = W.Workload(params=p, hf=hf, morphs=[m], inst_morph=np.zeros(1, np.int32),
                       ctrl=[W.sinusoid_controller(rng, max(m.n_joints, 0))],
                       pose=np.array([xyz + [1, 0, 0, 0]], np.float32))
        ow = O.OracleWorld(w)
        with N.World(w) as gw:
            res = run_windows(ow, gw, [0], starts=[0, 200])
        assert_windows(res, f"{m.name} dt={p.dt} K={p.K} mu={p.mu}", ow)


def _body(gw):
    return np.concatenate([gw.read_state(N.F_BODY).ravel(), gw.read_state(N.F_JOINT).ravel(),
                           gw.read_state(N.F_STEP).astype(np.float32).ravel()])


@pytest.mark.parametrize("six", [False, True])
def test_bitwise_chunking_graphs_and_persistence(six):
    """A trajectory does not depend on chunk length, hipGraph replay or the
    persistent queue (same lanes per robot): bit-identical states, with the
    ground-plane and the six-degree friction fit."""
    say(f"case: bitwise chunking / graphs / persistent, six-degree friction {six}")
    w = W.hexapod_batch(40, seed=11)
    w.params.friction_6dof = six
    out = []
    for chunk, graph, pers in ((100, 1, 0), (7, 0, 0), (33, 1, 1), (300, 0, 1)):
        with N.World(w) as gw:
            gw.set_launch(lanes_per_instance=32, chunk_steps=chunk, use_graph=graph,
                          persistent=pers, waves_per_cu=3)
            gw.step_n(150)
            gw.step_n(150)
            out.append(_body(gw))
    for o in out[1:]:
        np.testing.assert_array_equal(out[0], o)


def test_bitwise_batch_composition():
    """Instance results are the same alone or inside any batch."""
    say("case: bitwise batch composition")
    w = W.hexapod_batch(24, seed=12)
    with N.World(w) as gw:
        gw.set_launch(lanes_per_instance=16)
        gw.step_n(300)
        full = gw.read_state(N.F_BODY)
    for pick in ([5], [5, 0, 23], [23, 22, 21, 20, 19]):
        sub = W.subset(w, pick)
        with N.World(sub) as gs:
            gs.set_launch(lanes_per_instance=16)
            gs.step_n(300)
            part = gs.read_state(N.F_BODY)
        np.testing.assert_array_equal(part, full[:, pick])


def test_health_flag_isolates_instance():
    """A NaN written into one instance flags and freezes it; the others continue
    bit-identically to a clean run."""
    say("case: health isolation")
    w = W.hexapod_batch(8, seed=13)
    with N.World(w) as clean:
        clean.step_n(200)
        ref = clean.read_state(N.F_BODY)
    with N.World(w) as gw:
        om = gw.read_state(N.F_OMEGA)
        om[0, 3] = np.nan
        gw.write_state(N.F_OMEGA, om)
        gw.step_n(200)
        got = gw.read_state(N.F_BODY)
        flags = gw.read_state(N.F_FLAGS)
        steps = gw.read_state(N.F_STEP)
    assert flags[3] & 1 and steps[3] == 1
    others = [i for i in range(8) if i != 3]
    np.testing.assert_array_equal(got[:, others], ref[:, others])
    assert (flags[others] == 0).all() and (steps[others] == 200).all()
    # the oracle flags the same instance the same way
    ow = O.OracleWorld(w)
    st = ow.init_state(3)
    st[O.W_] = np.nan
    ow.run(3, st, 5)
    assert int(st[O.FLAGS]) & 1 and int(st[O.STEP]) == 1


def test_checkpoint_resume_is_exact():
    say("case: checkpoint/resume")
    w = W.hexapod_batch(12, seed=14)
    fields = [N.F_BODY, N.F_JOINT, N.F_JOINT_PREV, N.F_STEP, N.F_FLAGS, N.F_TELE]
    with N.World(w) as gw:
        gw.step_n(100)
        saved = {f: gw.read_state(f) for f in fields}
        gw.step_n(100)
        a = {f: gw.read_state(f) for f in fields}
        for f in fields:
            gw.write_state(f, saved[f])
        gw.step_n(100)
        b = {f: gw.read_state(f) for f in fields}
    for f in fields:
        np.testing.assert_array_equal(a[f], b[f])


def test_torch_stream_and_device_buffers():
    """Stepping on a torch stream and reading into a torch device tensor."""
    say("case: torch stream / device tensors")
    import torch
    w = W.hexapod_batch(10, seed=15)
    with N.World(w) as gw:
        s = torch.cuda.Stream()
        gw.step_n(50, stream=s)
        t = torch.empty((13, 10), dtype=torch.float32, device="cuda")
        gw.read_state(N.F_BODY, out=t)
        host = gw.read_state(N.F_BODY)
        np.testing.assert_array_equal(t.cpu().numpy(), host)
        ctrl = torch.zeros((10, gw.j_max, 3), dtype=torch.float32, device="cuda")
        gw.set_controller(ctrl)
        gw.step_n(10, stream=s)
        q = gw.read_state(N.F_JOINT)
        assert np.abs(q).max() == 0.0   # zero controller holds the joints at 0


def test_robot_built_with_construction_api():
    """A quadruped made with createBox/createCylinder/createJoint/rotateBody, stepped
    on the GPU from the tables npx_finalize_construction writes."""
    say("case: construction-API quadruped")
    b = N.MorphBuilder()
    torso = b.create_box(0.3, 0.05, 0.2, 0, 0, 0, 2.0)
    extra = b.create_sphere(0, 0, 0.04, 0.03, 0.3)
    b.connect_bodies(torso, extra)
    for hx in (-0.12, 0.12):
        for side in (-1, 1):
            hip = (hx, side * 0.1, 0.0)
            knee = (hx, side * 0.18, 0.0)
            upper = b.create_cylinder(*hip, *knee, 0.01, 0.15, ring_pts=8)
            lower = b.create_cylinder(*knee, hx, side * 0.18, -0.11, 0.01, 0.1, ring_pts=8)
            b.create_joint(torso, upper, (hx, side * 0.1, 0.0), (0, 0, 1))
            b.create_joint(upper, lower, (0, 0, 0.0), (1, 0, 0))   # anchor: upper's midpoint
    b.finalize_construction()
    m = b.tables("quadruped")
    rng = np.random.default_rng(4)
    ctrl = [W.sinusoid_controller(rng, m.n_joints)]
    w = W.Workload(params=W.Params(), hf=W.octave_terrain(5), morphs=[m],
                   inst_morph=np.zeros(1, np.int32), ctrl=ctrl,
                   pose=np.array([[0, 0, 0.16, 1, 0, 0, 0]], np.float32))
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, [0], starts=[0, 400])
    assert_windows(res, "construction-API quadruped", ow)


def test_force_weighted_friction_windows():
    """The friction fit weighted by each point's normal force (the refinement
    closing Sec. III-C): 32 hexapods on the terrain, 3 windows of 200 frames
    each against the oracle's weighted fit, and the weighting changes the
    trajectories."""
    say("case: force-weighted friction, 32 hexapods x 3 windows")
    w = W.hexapod_batch(32, seed=31, hf=W.octave_terrain(5), n_steps=600)
    w.params.friction_weighting = True
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, list(range(32)), starts=[0, 200, 400])
    assert_windows(res, "weighted", ow)
    w0 = W.hexapod_batch(32, seed=31, hf=W.octave_terrain(5), n_steps=600)
    with N.World(w) as gw_w, N.World(w0) as gw_u:
        gw_w.step_n(600)
        gw_u.step_n(600)
        d = np.abs(gw_w.read_state(N.F_COG)[:2] - gw_u.read_state(N.F_COG)[:2]).max()
    assert d > 1e-4, d


def test_six_dof_friction_windows():
    """The friction fit over the full rigid motion in 3-D (rotations about the
    other two axes as well, the refinement closing Sec. III-C): 32 hexapods on
    the terrain, 3 windows of 200 frames each against the oracle's six-degree
    fit, and the option changes the trajectories."""
    say("case: six-degree friction, 32 hexapods x 3 windows")
    w = W.hexapod_batch(32, seed=71, hf=W.octave_terrain(7), n_steps=600)
    w.params.friction_6dof = True
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, list(range(32)), starts=[0, 200, 400])
    assert_windows(res, "six-degree friction", ow)
    w0 = W.hexapod_batch(32, seed=71, hf=W.octave_terrain(7), n_steps=600)
    with N.World(w) as gw_6, N.World(w0) as gw_3:
        gw_6.step_n(600)
        gw_3.step_n(600)
        d = np.abs(gw_6.read_state(N.F_COG) - gw_3.read_state(N.F_COG)).max()
    assert d > 1e-4, d


def test_six_dof_uneven_bilinear_windows():
    """The six-degree fit on uneven random legged robots (legs that lie on the
    ground give contact sets close to a line) over the bilinear ground, at 32
    lanes per robot (two links per lane): 24 robots, 2 windows of 200 frames
    against the oracle."""
    say("case: six-degree + bilinear, 24 uneven robots x 2 windows")
    w = W.config3(seed=72, n_inst=24, n_steps=400)
    w.params.friction_6dof = True
    w.params.hf_bilinear = True
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        gw.set_launch(lanes_per_instance=32)
        res = run_windows(ow, gw, list(range(24)), starts=[0, 200])
    assert_windows(res, "six-degree uneven bilinear", ow)


def test_bilinear_ground_windows():
    """The height map read bilinearly between cell centres (the smoother-ground
    option): 32 hexapods on the terrain, 3 windows of 200 frames against the
    oracle's bilinear reading, and the reading changes the trajectories."""
    say("case: bilinear ground, 32 hexapods x 3 windows")
    w = W.hexapod_batch(32, seed=41, hf=W.octave_terrain(6), n_steps=600)
    w.params.hf_bilinear = True
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, list(range(32)), starts=[0, 200, 400])
    assert_windows(res, "bilinear", ow)
    w0 = W.hexapod_batch(32, seed=41, hf=W.octave_terrain(6), n_steps=600)
    with N.World(w) as gw_b, N.World(w0) as gw_t:
        gw_b.step_n(600)
        gw_t.step_n(600)
        d = np.abs(gw_b.read_state(N.F_COG)[:2] - gw_t.read_state(N.F_COG)[:2]).max()
    assert d > 1e-4, d


def test_paper_mode_on_terrain_windows():
    """The paper's operating point on the 2 cm terrain: 10 ms frames, joint
    targets every 8 frames (Sec. III-B), contacts softened to 150 N/m per point
    (stable at that frame length): 32 hexapods, 3 windows of 200 frames (2 s
    each) against the oracle."""
    say("case: paper mode on terrain, 32 hexapods x 3 windows")
    w = W.hexapod_batch(32, seed=51, n_steps=600)
    w.params.dt, w.params.K, w.params.k_n = 1e-2, 8, 150.0
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, list(range(32)), starts=[0, 200, 400])
    assert_windows(res, "paper mode", ow)


def test_joint_rate_limit_windows():
    """Joints turning at most 1 rad/s (the motors' speed, Sec. III-B) at the
    paper's operating point: 10 ms frames, joint targets every 8 frames,
    contacts at 150 N/m per point, on the terrain: 32 hexapods, 3 windows of
    200 frames (2 s each) against the oracle, and the limit changes the
    trajectories."""
    say("case: joint rate limit at 10 ms frames, 32 hexapods x 3 windows")
    w = W.hexapod_batch(32, seed=61, n_steps=600)
    w.params.dt, w.params.K, w.params.k_n, w.params.max_joint_rate = 1e-2, 8, 150.0, 1.0
    ow = O.OracleWorld(w)
    with N.World(w) as gw:
        res = run_windows(ow, gw, list(range(32)), starts=[0, 200, 400])
    assert_windows(res, "rate limit", ow)
    w0 = W.hexapod_batch(32, seed=61, n_steps=600)
    w0.params.dt, w0.params.K, w0.params.k_n = 1e-2, 8, 150.0
    with N.World(w) as gw_l, N.World(w0) as gw_u:
        gw_l.step_n(200)
        gw_u.step_n(200)
        d = np.abs(gw_l.read_state(N.F_JOINT) - gw_u.read_state(N.F_JOINT)).max()
    assert d > 1e-3, d
