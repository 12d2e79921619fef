"""Evolution of machine-code controllers (Sec. V): a population of 32-byte
programs for the interpreter of the command table drives hexapods with foot
contact sensors; every generation the best half is kept, duplicated and the
copies mutated (mutation is the only variation operator).

Every robot of a generation steps in one world on the GPU (npx_gp_run); this
module only draws programs, ranks them and keeps the loop.

Readings where the paper is silent:
  * programs start as uniformly random bytes; a mutation replaces each byte of
    a copy, independently with probability 1/32, by a uniformly random byte;
  * "selected, duplicated and mutated": the best 50 survive unchanged and
    their mutated copies take the other 50 places (the best never gets lost);
  * fitness is the distance walked along the robot's starting heading (+x)
    by its centre of gravity over the evaluation period;
  * every individual starts from the same pose on the same terrain, standing
    with all joint targets 0, program counter and accumulator 0;
  * the interpreter runs 16 instructions per joint update, a move command
    turns its motor by 0.05 rad, and every joint's range is +-0.8 rad (a
    hobby servo's; the hexapod's own joints are unlimited).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import native as N
from . import workloads as W

PROGRAM_BYTES = 32


def foot_links(m: W.Morph) -> list:
    """The leaf links of a morphology (the feet), in link order."""
    children = np.bincount(m.parent[1:], minlength=m.n_links) if m.n_links > 1 else np.zeros(1)
    return [int(l) for l in np.flatnonzero(children == 0)] if m.n_links > 1 else []


def random_programs(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.integers(0, 256, size=(n, PROGRAM_BYTES), dtype=np.uint8)


def mutate(programs: np.ndarray, rng: np.random.Generator, rate: float = 1.0 / 32) -> np.ndarray:
    out = programs.copy()
    hit = rng.random(out.shape) < rate
    out[hit] = rng.integers(0, 256, size=int(hit.sum()), dtype=np.uint8)
    return out


@dataclass
class GpConfig:
    seconds: float = 120.0      # evaluation period (two minutes of robot activity)
    dt: float = 1.0e-2          # the paper's frame
    K: int = 8                  # joint update every 80 ms
    k_n: float = 150.0          # contact stiffness stable at 10 ms frames
    n_instr: int = 16
    motor_step: float = 0.05
    servo_range: float = 0.8
    terrain_seed: int = 6


def servo_workload(w: W.Workload, cfg: GpConfig) -> W.Workload:
    """w at the controller's operating point: frames, stiffness, joint ranges
    of +-cfg.servo_range, standing commands (targets 0)."""
    w.params.dt, w.params.K, w.params.k_n = cfg.dt, cfg.K, cfg.k_n
    for m in w.morphs:
        m.joint[1:, 6] = -cfg.servo_range
        m.joint[1:, 7] = cfg.servo_range
    w.ctrl = [np.zeros_like(c) for c in w.ctrl]
    return w


def population_workload(n: int, cfg: GpConfig) -> W.Workload:
    """n hexapods at one start pose on the terrain, standing."""
    return servo_workload(W.hexapod_batch(n, seed=cfg.terrain_seed, spread=0.0), cfg)


def prepare(gw, w: W.Workload) -> None:
    """Foot sensors on the leaf links, and a step shape fixed by the population
    size (so that a kept program is re-evaluated bit for bit): with 8-frame
    launches, 64 lanes per robot below 1,024 robots and 32 from there on, the
    faster of the two in measured generations of 100 and of 4,096 robots."""
    gw.set_sensors(0, foot_links(w.morphs[0]))
    gw.set_launch(lanes_per_instance=64 if w.n_instances < 1024 else 32)


def evaluate(programs: np.ndarray, cfg: GpConfig, stream=None) -> np.ndarray:
    """Fitness of every program: +x distance of the CoG after cfg.seconds."""
    import torch
    n = programs.shape[0]
    w = population_workload(n, cfg)
    updates = int(round(cfg.seconds / (cfg.dt * cfg.K)))
    with N.World(w) as gw:
        prepare(gw, w)
        x0 = gw.read_state(N.F_COG)[0].astype(np.float64)
        prog = torch.as_tensor(programs, device="cuda")
        vm = torch.zeros((n, 2), dtype=torch.int32, device="cuda")
        targets = torch.zeros((n, max(gw.j_max, 1)), dtype=torch.float32, device="cuda")
        gw.gp_run(prog, vm, targets, updates, cfg.n_instr, cfg.motor_step, stream=stream)
        torch.cuda.synchronize()
        x1 = gw.read_state(N.F_COG)[0].astype(np.float64)
        flags = gw.read_state(N.F_FLAGS)
    fit = x1 - x0
    fit[flags != 0] = -np.inf      # a robot that blew up ranks last
    return fit


def evolve(generations: int, pop: int = 100, keep: int = 50, cfg: GpConfig | None = None,
           seed: int = 0, log=None):
    """The mutation-only loop; returns (final programs ranked, best fitness per
    generation, mean fitness per generation)."""
    cfg = cfg or GpConfig()
    rng = np.random.default_rng(seed)
    progs = random_programs(pop, rng)
    best, mean = [], []
    for g in range(generations):
        fit = evaluate(progs, cfg)
        order = np.argsort(-fit, kind="stable")
        progs = progs[order]
        fit = fit[order]
        best.append(float(fit[0]))
        mean.append(float(np.mean(fit[np.isfinite(fit)])) if np.isfinite(fit).any() else -np.inf)
        if log:
            log(f"generation {g}: best {best[-1]:.3f} m, mean {mean[-1]:.3f} m")
        if g + 1 < generations:
            parents = progs[:keep]
            progs = np.concatenate([parents, mutate(parents, rng)[:pop - keep]])
    return progs, best, mean
