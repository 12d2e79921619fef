"""Oracle of the evolved machine-code controller (Sec. V and its table of
interpreter commands): the interpreter, the foot contact sensors it reads and
the run of a program against the oracle's step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.

Readings where the paper is silent (each is stated again where it is used):
  * a program is 32 bytes, addresses 0..31 (jumps name one of 32 addresses);
    the program counter wraps from 31 to 0, so a program is an endless loop;
  * the accumulator is 8 bits wide: load puts the 5-bit value in it, read
    sensor puts 0 or 1, not inverts all 8 bits, inc and dec wrap modulo 256;
    jump if true jumps when it is non-zero;
  * the interpreter runs a fixed number of instructions at every joint update
    (every K frames) and keeps its program counter and accumulator between
    updates;
  * "move motor left/right" lowers/raises motor m's target angle by a fixed
    step, the target held within the joint's limits; motor m is joint m of
    the controller's order, a motor number past the last joint does nothing;
  * sensor s is the contact state of the s-th listed foot link: 1 when any
    of its mass points is in contact (strictly below the height of its cell,
    the step's own test), else 0; a sensor number past the list reads 0;
  * the targets reach the step as its commanded angles (a constant command
    A sin(2 pi 0 t + pi/2) = A per joint).
"""
from __future__ import annotations

import math

import numpy as np

OP_LEFT, OP_RIGHT, OP_SENSE, OP_LOAD, OP_JUMP, OP_NOT, OP_INC, OP_DEC = range(8)
PROGRAM_BYTES = 32


def interpret(prog, pc, acc, targets, sensors, n_instr, step, lo, hi):
    """Runs n_instr instructions of prog from (pc, acc). targets (float32 array,
    one per joint) is changed in place, each move by +-step (float32 sums) and
    then held within [lo, hi] (float32 per joint). Returns (pc, acc)."""
    step = np.float32(step)
    for _ in range(n_instr):
        byte = int(prog[pc])
        op, arg = byte >> 5, byte & 31
        nxt = (pc + 1) % PROGRAM_BYTES
        if op in (OP_LEFT, OP_RIGHT):
            if arg < len(targets):
                t = targets[arg] - step if op == OP_LEFT else targets[arg] + step
                targets[arg] = min(max(np.float32(t), lo[arg]), hi[arg])
        elif op == OP_SENSE:
            acc = int(sensors[arg]) if arg < len(sensors) else 0
        elif op == OP_LOAD:
            acc = arg
        elif op == OP_JUMP:
            if acc != 0:
                nxt = arg
        elif op == OP_NOT:
            acc = (~acc) & 0xFF
        elif op == OP_INC:
            acc = (acc + 1) & 0xFF
        else:
            acc = (acc - 1) & 0xFF
        pc = nxt
    return pc, acc


def sensors(ow, i, st, sensor_links):
    """Foot contact states of instance i at state st, and the smallest |H - z|
    over the sensed points (how far the closest decision is from flipping)."""
    m = ow.morph_of(i)
    P = ow.points(i, st)
    out = np.zeros(len(sensor_links), np.int32)
    margin = math.inf
    for s, link in enumerate(sensor_links):
        for k in np.flatnonzero(m.pt_link == link):
            d = ow.params.height(P[k, 0], P[k, 1]) - P[k, 2]
            margin = min(margin, abs(d))
            if d > 0.0:
                out[s] = 1
    return out, margin


def set_targets(ow, i, targets):
    """The targets as the oracle's controller of instance i: A = target, f = 0,
    phi = pi/2 (float32, as the library writes them)."""
    c = ow.ctrl[i]
    J = c.shape[0]
    c[:, 0] = targets[:J]
    c[:, 1] = 0.0
    c[:, 2] = np.float32(math.pi / 2)


def run(ow, i, st, prog, pc, acc, targets, sensor_links, n_updates, n_instr, step, lo, hi):
    """n_updates rounds of: sensors at the current state, n_instr instructions,
    the targets as commands, K frames of the oracle's step. Returns (pc, acc,
    smallest sensor margin seen)."""
    K = int(ow.w.params.K)
    margin = math.inf
    for _ in range(n_updates):
        s, mg = sensors(ow, i, st, sensor_links)
        margin = min(margin, mg)
        pc, acc = interpret(prog, pc, acc, targets, s, n_instr, step, lo, hi)
        set_targets(ow, i, targets)
        ow.run(i, st, K)
    return pc, acc, margin
