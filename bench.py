#!/usr/bin/env python3
"""Throughput benchmark: run-timesteps per second on one MI355X.

Workload: the two-pathway conflict network (one-hot inputs -> logistic
hidden layers -> 2-unit leaky competing accumulator), 64 control-gain
settings x 10,000 trials, step cap 1000, 100-bin decision-time histograms,
grid score with reward 1 and cost 0.1 and the best setting.  One sweep is:
output zero-fill, drive precompute, simulation with in-kernel histogram
reduction, score and argmax.  Inputs
are resident in HBM before timing starts.

Two arithmetic modes are timed back to back on the same inputs:
"FP32 batched" -- FP32 steps (normals and increments in float, accumulators
and threshold tests in double), the launch shape chosen by the autotuner,
and BATCH replicate sweeps of the workload (noise seeds 1..BATCH) in one
batched launch per benchmark step -- is the headline ``value``; a single
FP32 sweep per step is reported beside it, and "FP64 plain" is FP64
throughout, one sweep per step, default launch shape.

Also measured (same JSON line): the 256-unit rate network (65,536 runs, bf16
projections on matrix cores vs FP64), and the served mix -- Poisson arrivals
of sweeps of all model kinds and sizes, continuously batched under a memory
budget -- with p50/p99 latency and aggregate throughput.

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

# Lane-op slots of one run-step of the conflict-network LCA in the FP32-steps
# mode: the straight-line work the method needs per step, counted from the
# gfx950 instruction mix of the step body: Philox4x32-10 35 (what depends only
# on the run -- the round-1 product with the setting, the round-2 product with
# the trial-dependent word -- is done once per run; the step counter enters
# the first product as a scalar; the last round only the two low products the
# float normals use), Box-Muller 13 (two 24-bit uniforms, log, sqrt, sin, cos
# on the transcendental unit, scaling), the two-unit update 10 (three fused
# multiply-adds per unit, the float-to-double conversions and FP64
# accumulations), the near-threshold test 4 (the float images of the new
# state, which the next step needs anyway, a max and one compare; whether any
# lane is near is a scalar test).  Transcendentals count one slot.
LANE_OPS_PER_STEP = {"fp32_step": 62}

# "FP32 batched": this many replicate sweeps (noise seeds 1..BATCH) share one
# batched launch per benchmark step (the most one launch takes), so one
# sweep's tail of long runs overlaps the next sweep's work.
BATCH = 12

# HBM traffic of the simulation kernel from the profiler (FETCH_SIZE,
# WRITE_SIZE per dispatch, scaled by the same counters on a plain 1 GiB copy),
# valid only for the kernel sources it was measured on, and given per
# runs-per-lane (the number of workgroup flushes, hence the write traffic,
# depends on it).
TRAFFIC = {"sources_sha256": "eca0a96cb1cf47354afe1979d186ac3cf493f8d02cd39c4da3186237b32dfea4",
           "batch": 12,
           # profiles/sim_lane_lca_fp32_conflict_batched.md; key "runs_per_lane,block,tail_sweeps"
           "bytes_per_launch": {"4,512,0": 2838118, "6,512,0": 2294170, "8,512,0": 1897882,
                                "4,512,2": 3067904, "4,512,4": 3297690, "6,512,2": 2464154,
                                "6,512,4": 2637210, "8,512,2": 2054144, "8,512,4": 2211430}}
KERNEL_SOURCES = ("paper_2110_15425_amd/csrc/sim_lane.hip", "paper_2110_15425_amd/csrc/rng.hpp",
                  "paper_2110_15425_amd/csrc/lca_step.hpp", "paper_2110_15425_amd/csrc/internal.hpp",
                  "paper_2110_15425_amd/csrc/prep_score.hpp")


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _side(name):
    """(workload dict, launch kind) of a named side workload."""
    from paper_2110_15425_amd import workloads as W
    f32 = W.FP32_STEP
    table = {
        "c0_fp64": (W.ddm(), "launch"),
        "c0_fp32": (W.ddm(precision=f32), "launch"),
        "c0x1000_fp64": (W.ddm(trials=10_000_000), "launch"),
        "c0x1000_fp32": (W.ddm(trials=10_000_000, precision=f32), "launch"),
        "c1_fp64": (W.conflict(reward=1.0, cost=0.1), "launch"),
        "c1_fp32": (W.conflict(reward=1.0, cost=0.1, precision=f32), "launch"),
        "c2_fp32": (W.grid_search(precision=f32), "launch"),
        "c2_fp64": (W.grid_search(), "launch"),
        "c3_bf16": (W.rnn(precision=W.BF16_PROJ), "launch"),
        "c3_fp64": (W.rnn(), "launch"),
        "density_c0_64drifts": (W.ddm(drifts=[0.3 * (i + 1) / 64 for i in range(64)]), "density"),
        "density_c0_256drifts": (W.ddm(drifts=[0.3 * (i + 1) / 256 for i in range(256)]),
                                 "density"),
        "timecourse_c1_fp32": (W.conflict(precision=f32), "timecourse"),
        "loop_l8_m4_fp32": (W.control_loop(trials=20_000, costs=[0.0, 0.003, 0.01, 0.03],
                                           precision=f32), "launch"),
        "loop_l100_m1_fp32": (W.control_loop(trials=1000, levels=100, samples=1,
                                             costs=[0.0, 0.003, 0.01, 0.03], precision=f32),
                              "launch"),
        "unfused_c1_fp32": (W.conflict(precision=f32), "unfused"),
    }
    return table[name]


SIDE_WORKLOADS = ("c0_fp64", "c0_fp32", "c0x1000_fp64", "c0x1000_fp32", "c1_fp64", "c1_fp32",
                  "c2_fp32", "c2_fp64", "c3_bf16", "c3_fp64", "density_c0_64drifts",
                  "density_c0_256drifts",
                  "timecourse_c1_fp32", "loop_l8_m4_fp32", "loop_l100_m1_fp32",
                  "unfused_c1_fp32")


def side_workload(name, steps, warmup):
    """Time one named workload (default launch shape); returns its JSON dict."""
    import torch

    from paper_2110_15425_amd import cm
    w, how = _side(name)
    h = cm.Handle(0)
    ds = cm.DeviceSweep(h, w)
    if how == "density":
        out = torch.empty((int(w["n_settings"]), 2, int(w["max_steps"])), dtype=torch.float64,
                          device="cuda")
        m, s, keep = cm.structs(w, None, ds.grid.data_ptr())

        def launch():
            cm.check(cm.lib().cm_ddm_density(h.h, cm.C.byref(m), cm.C.byref(s), 1000, 1e-15,
                                             cm.C.c_void_p(out.data_ptr()),
                                             cm.C.c_void_p(torch.cuda.current_stream().cuda_stream)))
    elif how == "timecourse":
        def launch():
            ds.launch_timecourse(10)
    elif how == "unfused":
        def launch():
            ds.launch_unfused()
    else:
        launch = ds.launch
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    line = {"workload": name, "ms_per_step": ms, "steps": steps}
    if how != "density":
        rs = cm.run_steps(w, ds.results())
        line.update(run_steps=rs, run_steps_per_s=rs / (ms / 1e3))
    if name.startswith("loop_"):
        from paper_2110_15425_amd import workloads as W
        p = w["params"]
        per_step = int(p[W.LOOP_P["levels"]]) ** 2 * int(p[W.LOOP_P["samples"]])
        line["lookahead_evaluations_per_s"] = line["run_steps"] * per_step / (ms / 1e3)
    print(f"# {name}: {ms:.4f} ms/step", file=sys.stderr, flush=True)
    return line


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (used under the profiler)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no rate network, no served mix)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served-mix arrival window")
    ap.add_argument("--serve-queue-seconds", type=float, default=0.0,
                    help="also serve the mix this long with the conflict-network FP32 requests "
                         "through the device work queue (0: not run)")
    ap.add_argument("--workload", choices=sorted(SIDE_WORKLOADS), default=None,
                    help="time one other workload of the path instead (prints its own JSON "
                         "line; used to profile each kernel)")
    ap.add_argument("--oracle-table", action="store_true",
                    help="only time the FP64 CPU oracle on each configuration, one thread and "
                         "all threads (the CPU columns of the results table)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy five times (the reference "
                         "kernel that scales the profiler's FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--shape", default=None, metavar="RPL,SPS[,BLOCK[,WAVES[,TAIL]]]",
                    help="use this runs_per_lane,steps_per_sync (and workgroup size, register "
                         "cap, trailing sweeps in half-size chunks) for the batched launch "
                         "instead of tuning it (so that separate profiler runs see the same "
                         "kernel)")
    return ap.parse_args()


def time_mode(h, ds, steps, warmup):
    """ds: one DeviceSweep (cm_launch) or a list of them (one cm_launch_batch)."""
    import torch

    from paper_2110_15425_amd import cm

    def launch():
        if isinstance(ds, list):
            cm.launch_batch(h, ds)
        else:
            ds.launch()

    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    h.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    wall_ms = e0.elapsed_time(e1)
    sim_ms, n = h.profile_read()
    h.profile(False)
    return wall_ms, sim_ms / max(n, 1)


def time_graph(h, ds, steps, warmup):
    """Wall milliseconds of `steps` replays of the batched launch of ``ds``
    from the handle's graph cache (the first warm-up call captures it)."""
    import torch

    from paper_2110_15425_amd import cm
    for _ in range(max(1, warmup)):
        cm.launch_graph(h, ds)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        cm.launch_graph(h, ds)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def rate_network(cm, W):
    """The 256-unit rate network, 65,536 runs: bf16 projections vs FP64."""
    import torch
    out = {}
    h = cm.Handle(0)
    for name, prec in (("bf16_proj", W.BF16_PROJ), ("fp64", W.FP64)):
        w = W.rnn(precision=prec)
        ds = cm.DeviceSweep(h, w)
        wall_ms, kern_ms = time_mode(h, ds, 3, 1)
        rs = cm.run_steps(w, ds.results())
        out[name] = {"run_steps_per_s": rs * 3 / (wall_ms / 1e3), "ms_per_sweep": wall_ms / 3,
                     "kernel_ms": kern_ms, "run_steps": rs}
        print(f"# rate network {name}: {wall_ms / 3:.3f} ms/sweep, {rs} run-steps",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return out


def serving(cm, seconds, queue=False):
    """Served mix: Poisson(50/s) arrivals for `seconds`, continuously batched
    (with ``queue``: the conflict-network FP32 requests through the device
    work queue's persistent kernel, the rest through the slots)."""
    import numpy as np

    from paper_2110_15425_amd import serve
    n = max(8, int(50 * seconds))
    mix = serve.served_mix(n, rate_hz=50.0, seed=11)
    h = cm.Handle(0)
    warm = serve.served_mix(8, rate_hz=1e6, seed=12, max_runs=10_000)
    serve.run_mix(h, warm, queue=queue)
    steps_of = {}  # run-steps per request, taken as it finishes (its results are then released)
    done = serve.run_mix(h, mix, budget_bytes=32 << 30, n_streams=4, queue=queue,
                         on_done=lambda r: steps_of.__setitem__(r.rid, cm.run_steps(r.w, r.result)))
    steps = sum(steps_of.values())
    t0 = min(r.arrival for r in done)
    t1 = max(r.done for r in done)
    summ = serve.latency_summary(done)
    summ["by_config"] = serve.latency_by_config(done)
    summ.update({"arrival_rate_hz": 50.0, "window_s": float(mix[-1][0]),
                 "agg_run_steps_per_s": steps / (t1 - t0), "run_steps": int(steps),
                 "budget_gib": 32, "streams": 4, "device_queue": bool(queue),
                 "mean_runs_per_request": float(np.mean([r.w["n_settings"] * r.w["trials"]
                                                         for r in done]))})
    print(f"# serving: {summ}", file=sys.stderr, flush=True)
    return summ


def oracle_table():
    """The FP64 CPU oracle on each configuration with one thread and with all of
    this host's threads, on bounded samples (runs are independent, so the
    rate of a sample is the rate of the whole sweep)."""
    import oracle

    from paper_2110_15425_amd import workloads as W
    threads = len(os.sched_getaffinity(0))
    cases = [("c0", W.ddm(), W.ddm()),
             ("c1", W.conflict(), W.conflict(trials=1000)),
             ("c2", W.grid_search(), W.grid_search(trials=10)),
             ("c3", W.rnn(), W.rnn(trials=256))]
    rows = []
    for name, full, sample in cases:
        row = {"config": name, "sample_runs": int(sample["n_settings"] * sample["trials"]),
               "full_runs": int(full["n_settings"] * full["trials"])}
        for label, n in (("one_thread", 1), ("all_threads", threads)):
            small = sample
            if n == 1 and name in ("c3",):
                small = W.with_(sample, trials=32)
            t0 = time.perf_counter()
            rs, reps = 0, 0
            while reps == 0 or time.perf_counter() - t0 < 1.0:  # at least a second of work
                out = oracle.run(small, n_threads=n)
                rs += oracle.run_steps(small, out)
                reps += 1
            dt = time.perf_counter() - t0
            row[label] = {"run_steps_per_s": rs / dt, "seconds": dt, "repeats": reps,
                          "runs": int(small["n_settings"] * small["trials"])}
        row["threads"] = threads
        rows.append(row)
        print(f"# oracle {name}: 1 thread {row['one_thread']['run_steps_per_s']:.3e}, "
              f"{threads} threads {row['all_threads']['run_steps_per_s']:.3e} run-steps/s",
              file=sys.stderr, flush=True)
    return rows


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
                      f"({steps} run-steps, {dt:.2f} s wall on {threads} threads, "
                      f"{dt * threads:.0f} CPU-seconds)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(a sweep would shard by contiguous run ranges, one per GPU, with an "
              "all-reduce of the integer outputs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2110_15425_amd import cm, workloads as W

    if args.oracle_table:
        print(json.dumps({"oracle_table": oracle_table()}), flush=True)
        return
    if args.workload:
        print(json.dumps(side_workload(args.workload, args.steps, args.warmup)), flush=True)
        return
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
    from paper_2110_15425_amd import autotune

    w64 = W.conflict(reward=1.0, cost=0.1)
    w32 = W.with_(w64, precision=W.FP32_STEP)
    h_plain = cm.Handle(0)
    h_tuned = cm.Handle(0)
    # untimed: choose the FP32 launch shape on this device
    wb = [W.with_(w32, seed=1 + i) for i in range(BATCH)]
    if args.shape:
        rpl, sps, *rest = (int(v) for v in args.shape.split(","))
        h_tuned.set_tuning(W.LCA, W.FP32_STEP, runs_per_lane=rpl, steps_per_sync=sps,
                           block=rest[0] if rest else 256,
                           waves_per_simd=rest[1] if len(rest) > 1 else 0,
                           tail_sweeps=rest[2] if len(rest) > 2 else 0)
        tuned = h_tuned.get_tuning(W.LCA, W.FP32_STEP)
    else:
        tuned, _, _ = autotune.tune(h_tuned, wb, reps=2,
                                    candidates=[(r, s) for r in (4, 6, 8, 12, 16)
                                                for s in (8, 12, 16, 32)])
    h_single = cm.Handle(0)
    autotune.tune(h_single, w32, reps=2,
                  candidates=[(r, s) for r in (1, 2, 4) for s in (4, 8, 12, 16, 32)])
    res = {}
    for name, w, h in (("fp32_single", w32, h_single), ("fp64", w64, h_plain)):
        ds = cm.DeviceSweep(h, w)
        wall_ms, kern_ms = time_mode(h, ds, args.steps, args.warmup)
        out = ds.results()
        rs = cm.run_steps(w, out)
        res[name] = dict(run_steps=rs, wall_ms=wall_ms, kern_ms=kern_ms,
                         rate=rs * args.steps / (wall_ms / 1e3))
        print(f"# {name}: {wall_ms / args.steps:.4f} ms/sweep, simulation kernel "
              f"{kern_ms:.4f} ms, {rs} run-steps/sweep", file=sys.stderr, flush=True)
    # FP32 batched: BATCH replicate sweeps (noise seeds 1..BATCH) in one launch
    dsb = [cm.DeviceSweep(h_tuned, w) for w in wb]
    wall_ms, kern_ms = time_mode(h_tuned, dsb, args.steps, args.warmup)
    rs = sum(cm.run_steps(w, d.results()) for w, d in zip(wb, dsb))
    res["fp32_step"] = dict(run_steps=rs, wall_ms=wall_ms, kern_ms=kern_ms,
                            rate=rs * args.steps / (wall_ms / 1e3))
    print(f"# fp32 batched x{BATCH}: {wall_ms / args.steps:.4f} ms/step, simulation kernel "
          f"{kern_ms:.4f} ms, {rs} run-steps/step", file=sys.stderr, flush=True)
    # the same batched step replayed from the handle's graph cache; its
    # outputs must equal the eager launches'
    dsg = [cm.DeviceSweep(h_tuned, w) for w in wb]
    g_wall = time_graph(h_tuned, dsg, args.steps, args.warmup)
    g_same = all(np.array_equal(a.results()[k], b.results()[k])
                 for a, b in zip(dsg, dsb) for k in ("hist", "stats", "score", "best"))
    res["fp32_graph"] = dict(run_steps=rs, wall_ms=g_wall, rate=rs * args.steps / (g_wall / 1e3),
                             same=g_same)
    print(f"# fp32 batched x{BATCH} from a graph: {g_wall / args.steps:.4f} ms/step, "
          f"results {'equal' if g_same else 'DIFFERENT'}", file=sys.stderr, flush=True)

    head = res["fp32_step"]
    ach = head["run_steps"] * LANE_OPS_PER_STEP["fp32_step"] / (head["kern_ms"] / 1e3)
    # measured ceiling of the same step (random numbers + update, no tests,
    # refills or reductions) on this device
    ceil_rate = cm.ceiling(w32, handle=h_plain)
    kern_rate = head["run_steps"] / (head["kern_ms"] / 1e3)
    traffic = None
    if TRAFFIC["sources_sha256"] == sources_hash() and TRAFFIC["batch"] == BATCH:
        traffic = TRAFFIC["bytes_per_launch"].get(
            f"{tuned['runs_per_lane']},{tuned['block']},{tuned.get('tail_sweeps', 0)}")
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
                   "score": "reward 1.0, cost 0.1", "sweeps_per_step": BATCH,
                   "noise_seeds": f"1..{BATCH}", "run_steps_per_step": head["run_steps"],
                   "tuning": tuned},
        "fp32_single_sweep": {"value": res["fp32_single"]["rate"],
                              "ms_per_step": res["fp32_single"]["wall_ms"] / args.steps,
                              "kernel_ms": res["fp32_single"]["kern_ms"]},
        "fp32_batched_graph": {"value": res["fp32_graph"]["rate"],
                               "ms_per_step": res["fp32_graph"]["wall_ms"] / args.steps,
                               "results_equal_eager": res["fp32_graph"]["same"]},
        "fp64_plain": {"value": res["fp64"]["rate"],
                       "ms_per_step": res["fp64"]["wall_ms"] / args.steps,
                       "kernel_ms": res["fp64"]["kern_ms"]},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": ach / PEAK_LANE_OPS, "traffic": traffic,
                     "kernel": "sim_lane_kernel<LCA<FP32_STEP>>",
                     "kernel_ms": head["kern_ms"],
                     "lane_ops_per_run_step": LANE_OPS_PER_STEP["fp32_step"],
                     "measured_ceiling_run_steps_per_s": ceil_rate,
                     "frac_of_measured_ceiling": kern_rate / ceil_rate},
    }
    if not args.no_extras:
        line["rate_network"] = rate_network(cm, W)
        line["time_course"] = side_workload("timecourse_c1_fp32", 10, 2)
        line["closed_loop"] = side_workload("loop_l8_m4_fp32", 5, 1)
        line["serving"] = serving(cm, args.serve_seconds)
        if args.serve_queue_seconds > 0:
            line["serving_device_queue"] = serving(cm, args.serve_queue_seconds, queue=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w64)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
