"""Benchmark of the batched NeoPhysIx frame on one MI355X.

Workload: 4,096 18-DOF hexapods, each with its own seeded sinusoid controller,
on a shared 512x512 heightfield at 2 cm (four octaves, 3 cm amplitude), dt =
1 ms. One bench step is one frame of the whole hot path (detection, normal
forces, joint-angle determination, trial integration, friction least squares,
static-friction cap, correction) for every instance. Inputs are resident in
HBM before the timed region starts.

Prints one JSON line (rank 0): metric instance-steps/s, the dominant kernel's
roofline position (algorithmic FP32 FLOPs per launch over the launch time
measured with HIP events on the stream the kernel runs on) and the FP64 CPU
oracle timed on this host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12   # MI355X published FP32 vector FLOP/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.txt")
COPY_BYTES = 1 << 30   # plain device copy used to calibrate the HBM byte counters
KERNEL_SRC = os.path.join(ROOT, "paper_2411_05799_amd", "csrc", "step_kernel.hip")


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def pick_launch(gw, w, steps=50, stream=None):
    """Launch shape the bench times: the autotuner's fastest for this workload."""
    rec = gw.autotune(steps=steps, stream=stream)
    return rec


def measured_traffic(chunk, n_inst, lanes):
    """HBM bytes per launch from the committed rocprofv3 counter summary (lines
    "key: value"), if it was taken on the current kernel source at the same
    launch size and shape; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
        t = {k.strip(): v.strip() for k, v in t.items()}
        if (t.get("kernel_sha") != kernel_hash() or int(t.get("chunk_steps", -1)) != chunk
                or int(t.get("instances", -1)) != n_inst or int(t.get("lanes", -1)) != lanes):
            return None
        return float(t["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def copy_calibration():
    """One plain device-to-device copy of COPY_BYTES, for scaling FETCH_SIZE and
    WRITE_SIZE: run under rocprofv3 --pmc, the copy's counters must read COPY_BYTES."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES}), flush=True)


def cpu_baseline(w, n_inst, frames, threads):
    from oracle import oracle as O
    from paper_2411_05799_amd import workloads as W
    sub = W.subset(w, np.arange(n_inst))
    ow = O.OracleWorld(sub)
    states = ow.init_states()
    t0 = time.perf_counter()
    used = ow.run_batch(states, frames, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": n_inst * frames / dt, "unit": "instance-steps/s", "cores": int(used),
            "kind": "oracle",
            "sample": f"{n_inst} instances x {frames} frames of {w.name} "
                      f"(FP64 C oracle, OpenMP over instances, {used} threads, {dt:.2f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed frames")
    ap.add_argument("--warmup", type=int, default=200, help="untimed frames")
    ap.add_argument("--instances", type=int, default=4096)
    ap.add_argument("--cpu-instances", type=int, default=4096)
    ap.add_argument("--cpu-frames", type=int, default=250)
    ap.add_argument("--cpu-threads", type=int, default=int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes per robot (16/32/64); 0 = let the autotuner choose")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run the plain copy used to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.copy_calib:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the instances "
              "of a batch are independent, so a multi-GPU run would shard them with no "
              "per-frame exchange.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_05799_amd import native as N
    from paper_2411_05799_amd import workloads as W

    torch.cuda.init()
    w = W.config2(n_inst=args.instances, n_steps=args.steps)
    gw = N.World(w)
    stream = torch.cuda.Stream()
    if args.lanes:
        gw.set_launch(lanes_per_instance=args.lanes, persistent=args.persistent)
        tune = {"tried": []}
    else:
        tune = pick_launch(gw, w, stream=stream)
    launch = gw.get_launch().as_dict()
    chunk = launch["chunk_steps"]

    gw.step_n(args.warmup, stream=stream)
    stream.synchronize()
    torch.cuda.synchronize()

    # timed region: HIP events between chunk launches on the kernel's own stream
    n_chunks = (args.steps + chunk - 1) // chunk
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_chunks + 1)]
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev[0].record(stream)
        left = args.steps
        for k in range(n_chunks):
            c = min(chunk, left)
            gw.step_n(c, stream=stream)
            ev[k + 1].record(stream)
            left -= c
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(n_chunks)]
    total_ms = ev[0].elapsed_time(ev[-1])
    flags = gw.read_state(N.F_FLAGS)

    I = w.n_instances
    value = I * args.steps / (total_ms * 1e-3)
    flops_frame = gw.flops_per_step()            # summed over instances, one frame
    full = [ms for k, ms in enumerate(launch_ms) if (k + 1) * chunk <= args.steps]
    avg_ms = float(np.mean(full)) if full else float(np.mean(launch_ms))
    achieved = flops_frame * chunk / (avg_ms * 1e-3)
    traffic = measured_traffic(chunk, I, launch["lanes_per_instance"])

    out = {
        "metric": "instance-steps/s",
        "value": value,
        "unit": "instance-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": I, "frames": args.steps, "dt_s": 1e-3,
                   "points_per_robot": int(w.morphs[0].n_points),
                   "links_per_robot": int(w.morphs[0].n_links),
                   "heightfield": f"{w.hf.nx}x{w.hf.ny} @ {1 / w.hf.s:.3f} m",
                   "launch": launch, "flagged_instances": int((flags != 0).sum())},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
                     "traffic": traffic,
                     "kernel": "step_kernel", "launch_ms": avg_ms,
                     "flops_per_launch": flops_frame * chunk,
                     "frames_per_launch": chunk, "launches": len(launch_ms)},
        "wall_s": wall,
        "autotune": tune["tried"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, min(args.cpu_instances, I), args.cpu_frames,
                                           args.cpu_threads)
    gw.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
