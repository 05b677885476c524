#!/usr/bin/env python3
"""Throughput benchmark: run-timesteps per second on one MI355X.

Workload: the two-pathway conflict network (one-hot inputs -> logistic
hidden layers -> 2-unit leaky competing accumulator), 64 control-gain
settings x 10,000 trials, step cap 1000, 100-bin decision-time histograms,
grid score with reward 1 and cost 0.1 and the best setting.  One step of the
benchmark is one whole sweep: output zero-fill, drive precompute,
simulation with in-kernel histogram reduction, score and argmax.  Inputs
are resident in HBM before timing starts.

Two arithmetic modes are timed back to back on the same inputs:
FP32 steps (normals and increments in float, accumulators and threshold
tests in double) -- the headline ``value`` -- and FP64 throughout.

Printed: one JSON line.  ``roofline`` describes the simulation kernel (the
dominant kernel) against the chip's VALU issue rate; ``cpu_baseline`` is the
FP64 CPU oracle on this host's cores over the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz,
# counted in 32-bit lane-operation slots (a wave64 full-rate instruction takes
# 64 slots, a quarter-rate one 256).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# Lane-op slots of one run-step of the conflict-network LCA, by mode: the
# straight-line work the method needs per step (one Philox4x32-10 block, a
# Box-Muller pair, the two-unit update and threshold tests), counted from the
# instruction mix of the step body and weighted by issue rate.  Derivation
# in DESIGN.md ("Roofline accounting").
LANE_OPS_PER_STEP = {"fp32_step": 176, "fp64": 352}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (used under the profiler)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy five times (the reference "
                         "kernel that scales the profiler's FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


def time_mode(h, ds, steps, warmup):
    import torch
    for _ in range(warmup):
        ds.launch()
    torch.cuda.synchronize()
    h.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ds.launch()
    e1.record()
    torch.cuda.synchronize()
    wall_ms = e0.elapsed_time(e1)
    sim_ms, n = h.profile_read()
    h.profile(False)
    return wall_ms, sim_ms / max(n, 1)


def cpu_baseline(w):
    """The FP64 oracle on this host: the same sweep, all cores."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    reps, steps = 0, 0
    while True:
        out = oracle.run(w, n_threads=threads)
        steps += oracle.run_steps(w, out)
        reps += 1
        if time.perf_counter() - t0 > 1.5 or reps >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": steps / dt, "unit": "run-timesteps/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} full sweep(s) of the same workload in FP64 "
                      f"({steps} run-steps, {dt:.2f} s wall)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(runs shard by setting range across GPUs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2110_15425_amd import cm, workloads as W

    if args.calibrate_copy:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 5}))
        return
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w64 = W.conflict(reward=1.0, cost=0.1)
    w32 = W.with_(w64, precision=W.FP32_STEP)
    h = cm.Handle(0)
    res = {}
    for name, w in (("fp32_step", w32), ("fp64", w64)):
        ds = cm.DeviceSweep(h, w)
        wall_ms, kern_ms = time_mode(h, ds, args.steps, args.warmup)
        out = ds.results()
        rs = cm.run_steps(w, out)
        res[name] = dict(run_steps=rs, wall_ms=wall_ms, kern_ms=kern_ms,
                         rate=rs * args.steps / (wall_ms / 1e3))
        print(f"# {name}: {wall_ms / args.steps:.4f} ms/sweep, simulation kernel "
              f"{kern_ms:.4f} ms, {rs} run-steps/sweep", file=sys.stderr, flush=True)

    head = res["fp32_step"]
    ach = head["run_steps"] * LANE_OPS_PER_STEP["fp32_step"] / (head["kern_ms"] / 1e3)
    line = {
        "metric": "run-timesteps/sec on 1 MI355X (FP32 batched vs FP64 plain)",
        "value": head["rate"],
        "unit": "run-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["wall_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 steps / f64 accumulators",
        "data": "synthetic (seeded weights U(-2,2), Philox noise)",
        "config": {"workload": "conflict network -> LCA, 64 control settings x 10000 trials",
                   "settings": 64, "trials": 10000, "max_steps": 1000, "n_bins": 100,
                   "score": "reward 1.0, cost 0.1", "run_steps_per_sweep": head["run_steps"]},
        "fp64_plain": {"value": res["fp64"]["rate"], "ms_per_step": res["fp64"]["wall_ms"] / args.steps,
                       "kernel_ms": res["fp64"]["kern_ms"]},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": ach / PEAK_LANE_OPS, "traffic": None,
                     "kernel": "sim_lane_kernel<LCA<FP32_STEP>>",
                     "kernel_ms": head["kern_ms"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w64)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
