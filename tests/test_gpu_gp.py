"""The machine-code controller on the GPU (npx_gp_run) vs the oracle, through
the C ABI.

The interpreter is integer and byte work, its targets float32 sums of the
motor step: program counter, accumulator and targets must match the oracle
bit for bit, given the same sensor readings. The sensors are contact
decisions taken on float32 points (GPU) and float64 points (oracle) of the
same state; an instance whose closest sensed point lies within 1e-5 m of the
ground at an update could read either way and is not compared (at most 20%).
Bodies: 1e-4 m over 200-frame windows, as the step's own windows.
"""
import sys

import numpy as np
import pytest

from oracle import gp_oracle as G
from oracle import oracle as O
from paper_2411_05799_amd import gp as GP
from paper_2411_05799_amd import native as N
from paper_2411_05799_amd import workloads as W

from _helpers import POS_TOL, gpu_available, read_states

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")]

MARGIN = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _world(n, seed):
    """n hexapods spread over the terrain at the controller's operating point."""
    return GP.servo_workload(W.hexapod_batch(n, seed=seed), GP.GpConfig())


def _limits(m):
    return m.joint[1:, 6].astype(np.float32), m.joint[1:, 7].astype(np.float32)


def _warm(gw, n, rng):
    """Random programs run for 10 updates, so legs swing and feet lift."""
    import torch
    progs = torch.as_tensor(GP.random_programs(n, rng), device="cuda")
    vm = torch.zeros((n, 2), dtype=torch.int32, device="cuda")
    tg = torch.zeros((n, gw.j_max), dtype=torch.float32, device="cuda")
    gw.gp_run(progs, vm, tg, 10, 16, 0.05)
    torch.cuda.synchronize()
    return progs, vm, tg


def test_one_update_matches_oracle_bit_for_bit():
    """64 hexapods with random programs: after 10 updates, one more update on
    both sides from the same state, program counters, accumulators and targets
    equal; the sensor readings seen cover both values."""
    say("case: gp / one update, 64 hexapods")
    import torch
    n = 64
    w = _world(n, seed=12)
    m = w.morphs[0]
    feet = GP.foot_links(m)
    lo, hi = _limits(m)
    ow = O.OracleWorld(w)
    J = m.n_links - 1
    with N.World(w) as gw:
        gw.set_sensors(0, feet)
        progs, vm, tg = _warm(gw, n, np.random.default_rng(4))
        states = read_states(gw, range(n), lambda i: J)
        vm0, tg0, p = vm.cpu().numpy(), tg.cpu().numpy(), progs.cpu().numpy()
        gw.gp_run(progs, vm, tg, 1, 24, 0.05)
        torch.cuda.synchronize()
        vm1, tg1 = vm.cpu().numpy(), tg.cpu().numpy()
    compared, seen = 0, set()
    for i in range(n):
        s, margin = G.sensors(ow, i, states[i], feet)
        if margin < MARGIN:
            continue
        seen.update(int(v) for v in s)
        t = tg0[i, :J].copy()
        pc, acc = G.interpret(p[i], int(vm0[i, 0]), int(vm0[i, 1]), t, s, 24, 0.05, lo, hi)
        assert (pc, acc) == (int(vm1[i, 0]), int(vm1[i, 1])), i
        assert np.array_equal(t, tg1[i, :J]), i
        compared += 1
    say(f"  compared {compared} of {n}, sensor values seen {sorted(seen)}")
    assert compared >= 0.8 * n and seen == {0, 1}


def test_windows_match_oracle():
    """16 hexapods, 25 updates (200 frames, 2 s) from the same state on both
    sides: controller state bit for bit and bodies within 1e-4 m, for every
    instance whose sensed points never came within 1e-5 m of the ground."""
    say("case: gp / 25-update windows, 16 hexapods")
    import torch
    n = 16
    w = _world(n, seed=13)
    m = w.morphs[0]
    feet = GP.foot_links(m)
    lo, hi = _limits(m)
    ow = O.OracleWorld(w)
    J = m.n_links - 1
    with N.World(w) as gw:
        gw.set_sensors(0, feet)
        progs, vm, tg = _warm(gw, n, np.random.default_rng(5))
        states = read_states(gw, range(n), lambda i: J)
        vm0, tg0, p = vm.cpu().numpy(), tg.cpu().numpy(), progs.cpu().numpy()
        gw.gp_run(progs, vm, tg, 25, 16, 0.05)
        torch.cuda.synchronize()
        vm1, tg1 = vm.cpu().numpy(), tg.cpu().numpy()
        cog = gw.read_state(N.F_COG)
    compared = 0
    for i in range(n):
        st = states[i].copy()
        t = tg0[i, :J].copy()
        pc, acc, margin = G.run(ow, i, st, p[i], int(vm0[i, 0]), int(vm0[i, 1]), t, feet, 25, 16,
                                0.05, lo, hi)
        if margin < MARGIN:
            continue
        compared += 1
        assert (pc, acc) == (int(vm1[i, 0]), int(vm1[i, 1])), i
        assert np.array_equal(t, tg1[i, :J]), i
        err = np.abs(st[:3] - cog[:, i]).max()
        assert err <= POS_TOL, (i, err)
    say(f"  compared {compared} of {n}")
    assert compared >= 0.6 * n


def test_evolution_keeps_its_best_and_refuses_bad_calls():
    """Three generations of 32 programs (4 s each): the best fitness never
    drops (the kept half is re-evaluated bit for bit in a new batch), and the
    entry points refuse bad arguments."""
    say("case: gp / evolution loop, errors")
    cfg = GP.GpConfig(seconds=4.0)
    progs, best, mean = GP.evolve(3, pop=32, keep=16, cfg=cfg, seed=1, log=say)
    assert all(b1 >= b0 for b0, b1 in zip(best, best[1:])), best
    assert np.isfinite(best[-1])

    import torch
    w = _world(4, seed=1)
    with N.World(w) as gw:
        prog = torch.zeros((4, 32), dtype=torch.uint8, device="cuda")
        vm = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
        with pytest.raises(N.NpxError):
            gw.gp_run(prog, vm, torch.zeros((4, gw.j_max - 1), device="cuda"), 1, 16, 0.05)
        tg = torch.zeros((4, gw.j_max), device="cuda")
        with pytest.raises(N.NpxError):
            gw.gp_run(prog, vm, tg, 1, 5000, 0.05)
        with pytest.raises(N.NpxError):
            gw.gp_run(prog, vm, tg, 1, 16, float("nan"))
        with pytest.raises(N.NpxError):
            gw.set_sensors(0, [w.morphs[0].n_links])
        with pytest.raises(N.NpxError):
            gw.set_sensors(0, list(range(33)))
        # without sensors every sensor reads 0: "read sensor 0; jump 0 if true;
        # motor 0 right" turns motor 0 once per pass
        prog[:, 0] = (2 << 5) | 0
        prog[:, 1] = (4 << 5) | 0
        prog[:, 2] = (1 << 5) | 0
        prog[:, 3:] = (4 << 5) | 0      # jump 0 (accumulator 0: falls through)
        gw.gp_run(prog, vm, tg, 1, 32, 0.05)
        torch.cuda.synchronize()
        assert np.allclose(tg[:, 0].cpu().numpy(), np.float32(0.05))
        assert np.all(vm.cpu().numpy()[:, 0] == 0)


def test_targets_controller_kind():
    """npx_set_controller with joint targets: after the next joint update the
    joints sit exactly at the targets held within their limits, from host and
    device targets alike, and the trajectory equals the one driven by the
    equivalent sinusoid rows (target, 0, pi/2) bit for bit."""
    say("case: controller kind targets")
    import math
    import torch
    w = _world(8, seed=2)
    m = w.morphs[0]
    lo, hi = _limits(m)
    rng = np.random.default_rng(6)
    with N.World(w) as ga, N.World(w) as gb, N.World(w) as gc:
        J = ga.j_max
        t = rng.uniform(-1.0, 1.0, (8, J)).astype(np.float32)
        ga.set_targets(t)
        gb.set_targets(torch.as_tensor(t, device="cuda"))
        rows = np.stack([t, np.zeros_like(t), np.full_like(t, np.float32(math.pi / 2))], axis=-1)
        gc.set_controller(rows)
        for g in (ga, gb, gc):
            g.step_n(1)
        want = np.clip(t, lo[None, :J], hi[None, :J]).T
        for g in (ga, gb, gc):
            assert np.array_equal(g.read_state(N.F_JOINT), want)
        for g in (ga, gb, gc):
            g.step_n(49)
        body = [g.read_state(N.F_BODY) for g in (ga, gb, gc)]
        assert np.array_equal(body[0], body[1]) and np.array_equal(body[0], body[2])
        with pytest.raises(N.NpxError):
            ga.set_targets(t[:, :-1])


def test_graph_blocks_equal_single_launches():
    """Updates replayed from captured blocks of 25 equal updates launched one by
    one, bit for bit (60 updates: two blocks and a remainder), also after the
    controller's buffers and the sensor tables change (fresh capture)."""
    say("case: gp / captured update blocks")
    import torch
    n = 24
    w = _world(n, seed=21)
    feet = GP.foot_links(w.morphs[0])
    progs = torch.as_tensor(GP.random_programs(n, np.random.default_rng(8)), device="cuda")
    out = []
    for graph in (1, 0):
        with N.World(w) as gw:
            gw.set_sensors(0, feet)
            gw.set_launch(use_graph=graph)
            res = []
            for rep in range(2):
                vm = torch.zeros((n, 2), dtype=torch.int32, device="cuda")
                tg = torch.zeros((n, gw.j_max), dtype=torch.float32, device="cuda")
                gw.gp_run(progs, vm, tg, 60, 16, 0.05)
                torch.cuda.synchronize()
                res += [vm.cpu().numpy(), tg.cpu().numpy(), gw.read_state(N.F_BODY)]
                gw.set_sensors(0, feet[:3])
            out.append(res)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
