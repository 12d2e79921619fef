"""Pins of the machine-code controller oracle (Sec. V, its table of interpreter
commands): hand-traced programs for every command, the wrap of the program
counter and the 8-bit accumulator, motor steps held at the joint limits, the
foot contact sensors of a standing and a lifted robot, and the targets
reaching the step as its commanded angles."""
import math

import numpy as np

from oracle import gp_oracle as G
from oracle import oracle as O
from paper_2411_05799_amd import workloads as W


def op(code, arg=0):
    return (code << 5) | arg


def prog(*ops):
    p = np.full(32, op(G.OP_LOAD, 0), np.uint8)
    p[:len(ops)] = ops
    return p


LO = np.full(4, -0.25, np.float32)
HI = np.full(4, 0.25, np.float32)


def test_countdown_loop_then_motor():
    # 0 load 3; 1 dec; 2 jump-if-true 1; 3 motor 0 right; 4.. load 0
    p = prog(op(G.OP_LOAD, 3), op(G.OP_DEC), op(G.OP_JUMP, 1), op(G.OP_RIGHT, 0))
    t = np.zeros(4, np.float32)
    # executed: 0 1 2 1 2 1 2 3 4 -> pc 5, acc 0, one step right
    pc, acc = G.interpret(p, 0, 0, t, [], 9, 0.1, LO, HI)
    assert (pc, acc) == (5, 0)
    assert t[0] == np.float32(0.1) and np.all(t[1:] == 0)


def test_accumulator_is_eight_bits():
    pc, acc = G.interpret(prog(op(G.OP_LOAD, 0), op(G.OP_NOT)), 0, 0, np.zeros(1, np.float32),
                          [], 2, 0.1, LO, HI)
    assert (pc, acc) == (2, 255)
    pc, acc = G.interpret(prog(op(G.OP_LOAD, 0), op(G.OP_NOT), op(G.OP_INC)), 0, 0,
                          np.zeros(1, np.float32), [], 3, 0.1, LO, HI)
    assert (pc, acc) == (3, 0)
    pc, acc = G.interpret(prog(op(G.OP_LOAD, 0), op(G.OP_DEC)), 0, 0, np.zeros(1, np.float32),
                          [], 2, 0.1, LO, HI)
    assert acc == 255
    pc, acc = G.interpret(prog(op(G.OP_LOAD, 5), op(G.OP_NOT)), 0, 0, np.zeros(1, np.float32),
                          [], 2, 0.1, LO, HI)
    assert acc == 250


def test_program_counter_wraps_and_state_carries_over():
    p = np.full(32, op(G.OP_INC), np.uint8)
    pc, acc = G.interpret(p, 0, 0, np.zeros(1, np.float32), [], 40, 0.1, LO, HI)
    assert (pc, acc) == (8, 40)
    pc, acc = G.interpret(p, pc, acc, np.zeros(1, np.float32), [], 30, 0.1, LO, HI)
    assert (pc, acc) == (6, 70)


def test_sensors_and_conditional_jump():
    p = prog(op(G.OP_SENSE, 1), op(G.OP_JUMP, 7), op(G.OP_SENSE, 9), op(G.OP_JUMP, 20))
    pc, acc = G.interpret(p, 0, 0, np.zeros(1, np.float32), [0, 1, 0], 2, 0.1, LO, HI)
    assert (pc, acc) == (7, 1)
    pc, acc = G.interpret(p, 0, 0, np.zeros(1, np.float32), [1, 0, 1], 2, 0.1, LO, HI)
    assert (pc, acc) == (2, 0)
    # a sensor past the list reads 0: no jump
    pc, acc = G.interpret(p, 2, 9, np.zeros(1, np.float32), [1, 1, 1], 2, 0.1, LO, HI)
    assert (pc, acc) == (4, 0)


def test_motor_steps_held_at_limits_and_unknown_motors_ignored():
    p = np.full(32, op(G.OP_LEFT, 2), np.uint8)
    p[3] = op(G.OP_RIGHT, 30)
    t = np.zeros(4, np.float32)
    G.interpret(p, 0, 0, t, [], 2, 0.1, LO, HI)
    assert t[2] == np.float32(np.float32(0) - np.float32(0.1)) - np.float32(0.1)
    G.interpret(p, 2, 0, t, [], 2, 0.1, LO, HI)   # motor 30 (no such joint), then left
    assert t[2] == np.float32(-0.25) and np.all(t[[0, 1, 3]] == 0)


def _hexapod(z):
    w = W.hexapod_batch(1, seed=3, hf=W.flat_ground())
    w.pose[0, :3] = [0.0, 0.0, z]
    return w


def _feet(m):
    children = np.bincount(m.parent[1:], minlength=m.n_links)
    return [int(l) for l in np.flatnonzero(children == 0)]


def test_foot_sensors_standing_and_lifted():
    w = _hexapod(0.15)
    ow = O.OracleWorld(w)
    feet = _feet(w.morphs[0])
    assert len(feet) == 6
    st = ow.init_state(0)
    G.set_targets(ow, 0, np.zeros(18, np.float32))
    ow.run(0, st, 1500)                      # settles on its feet
    s, margin = G.sensors(ow, 0, st, feet)
    assert np.all(s == 1) and margin >= 0.0
    w2 = _hexapod(1.0)
    ow2 = O.OracleWorld(w2)
    s2, margin2 = G.sensors(ow2, 0, ow2.init_state(0), feet)
    assert np.all(s2 == 0) and margin2 > 0.5


def test_targets_become_the_commanded_angles():
    """After one update the joints sit at the targets (held within limits)."""
    w = _hexapod(1.0)
    ow = O.OracleWorld(w)
    st = ow.init_state(0)
    targets = np.linspace(-0.3, 0.3, 18).astype(np.float32)
    lo = w.morphs[0].joint[1:, 6].astype(np.float32)
    hi = w.morphs[0].joint[1:, 7].astype(np.float32)
    pc, acc, _ = G.run(ow, 0, st, prog(), 0, 0, targets, _feet(w.morphs[0]), 1, 4, 0.05, lo, hi)
    q = st[O.HDR:O.HDR + 18]
    want = np.clip(targets.astype(np.float64), lo, hi)
    assert np.abs(q - want).max() < 1e-12
    assert (pc, acc) == (4, 0)
