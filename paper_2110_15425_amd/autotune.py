"""Launch-shape autotuner for libcm sweeps.

For a given workload it times the simulation kernel (HIP events that libcm
records around it) for each candidate launch shape and keeps the fastest.
The knobs are the ones in ``cm_tuning``: runs handed to a workgroup per lane
(which trades occupancy against the tail of long runs), steps between
refills of finished lanes (which trades idle lanes against refill cost) and,
for the lane kernels, the workgroup size (how many unfinished runs one
workgroup packs together while its chunk drains), the register cap that
sets how many wavefronts fit per SIMD (the register use versus occupancy
trade-off of the paper's GPU kernels: more wavefronts hide more latency, but
a cap below the kernel's own register use spills) and, for batched
launches, half-size chunks for the last sweeps (a shorter launch tail).
Results can be persisted in a JSON cache keyed by device, kind, precision
and a size class of the sweep, so a later process reuses them without
re-timing.

Integer outputs do not depend on the launch shape (random streams are keyed
by run, reductions are integer), so tuning never changes results.
"""
import json
import math
import os

from . import cm

RUNS_PER_LANE = (1, 2, 4, 6, 8, 12, 16, 32)
STEPS_PER_SYNC = (2, 4, 8, 12, 16, 32)
RUNS_PER_WAVE = (1, 2, 4, 8, 16, 32, 64)  # DDM, one wavefront per run
WAVES_PER_SIMD = (0, 4, 8)  # 0: the compiler's register allocation
BLOCKS = (256, 512, 1024)  # threads per workgroup of the lane kernels
TAIL_SWEEPS = (0, 2, 4)  # batched launches: trailing sweeps in half-size chunks


def size_class(w):
    """Coarse key: log2 buckets of settings, trials and step cap."""
    b = lambda v: int(math.log2(max(1, int(v))))  # noqa: E731
    return f"S{b(w['n_settings'])}-T{b(w['trials'])}-N{b(w['max_steps'])}"


def cache_key(w, device_name):
    return f"{device_name}|k{int(w['kind'])}|p{int(w['precision'])}|{size_class(w)}"


def time_shape(handle, ds, reps=3):
    """Mean simulation-kernel milliseconds over reps launches (after one
    warm-up); ``ds`` is a DeviceSweep or a list of them (one batched launch)."""
    import torch

    def launch():
        if isinstance(ds, list):
            cm.launch_batch(handle, ds)
        else:
            ds.launch()

    launch()
    torch.cuda.synchronize()
    handle.profile(True)
    for _ in range(reps):
        launch()
    ms, n = handle.profile_read()
    handle.profile(False)
    return ms / max(n, 1)


def default_candidates(w):
    """(runs_per_lane, steps_per_sync, lanes_per_run) shapes worth timing."""
    c = [(r, s, 1) for r in RUNS_PER_LANE for s in STEPS_PER_SYNC]
    if int(w["kind"]) == 0:  # DDM: also one wavefront per run
        c += [(r, 4, 64) for r in RUNS_PER_WAVE]
    return c


def tune(handle, w, reps=3, candidates=None, verbose=False, finalists=4, rounds=3):
    """Time every candidate shape on workload ``w`` (a workload dict, or a list
    of workloads of one kind and precision timed as one batched launch);
    install and return the best as (tuning dict, kernel ms, table).  Table
    rows are (rpl, sps, lpr, ms, waves cap, block, tail sweeps): first every
    candidate shape in 256-thread workgroups, then, for the lane kernels,
    the best shape in workgroups of 512 and 1024 threads (with as many and
    with half as many runs per lane), then the register caps on the best of
    those, then -- for a batched launch -- half-size chunks for its last
    sweeps.
    Shapes within a few per cent of each other are not told apart by one
    timing, so the ``finalists`` fastest are timed ``rounds`` more times and
    ranked by their fastest timing."""
    ws = w if isinstance(w, list) else [w]
    w = ws[0]
    kind, prec = int(w["kind"]), int(w["precision"])
    ds = [cm.DeviceSweep(handle, x) for x in ws] if len(ws) > 1 else cm.DeviceSweep(handle, w)
    table = []
    cands = candidates or default_candidates(w)

    def run(rpl, sps, lpr, waves=0, block=256, best_of=1, tail=0):
        handle.set_tuning(kind, prec, runs_per_lane=rpl, steps_per_sync=sps, lanes_per_run=lpr,
                          waves_per_simd=waves, block=block, tail_sweeps=tail)
        return min(time_shape(handle, ds, reps) for _ in range(best_of))

    for c in cands:
        rpl, sps = c[0], c[1]
        lpr = c[2] if len(c) > 2 else 1
        ms = run(rpl, sps, lpr)
        table.append((rpl, sps, lpr, ms, 0, 256, 0))
        if verbose:
            print(f"  runs/lane {rpl:3d} steps/sync {sps:3d} lanes/run {lpr:2d}: {ms:.4f} ms",
                  flush=True)
    table.sort(key=lambda r: r[3])
    for i, (rpl, sps, lpr, ms, _, _, _) in enumerate(table[:finalists]):
        ms = min(ms, run(rpl, sps, lpr, best_of=rounds))
        table[i] = (rpl, sps, lpr, ms, 0, 256, 0)
    best = min(table, key=lambda r: r[3])
    rpl, sps, lpr, ms, _, _, _ = best
    if kind in (0, 1) and lpr != 64:
        # workgroup size: a larger workgroup packs more unfinished runs
        # together while its chunk drains, but holds more of a compute unit
        for blk in BLOCKS[1:]:
            for r in sorted({rpl, max(1, rpl // 2)}):
                t = run(r, sps, lpr, block=blk, best_of=rounds)
                table.append((r, sps, lpr, t, 0, blk, 0))
                if verbose:
                    print(f"  block {blk} runs/lane {r}: {t:.4f} ms", flush=True)
        best = min(table, key=lambda r: r[3])
        # the occupancy axis, on the best shape: registers capped for 4 or 8
        # wavefronts per SIMD against the compiler's own allocation
        for wv in WAVES_PER_SIMD[1:]:
            t = run(best[0], sps, lpr, waves=wv, block=best[5], best_of=rounds)
            table.append((best[0], sps, lpr, t, wv, best[5], 0))
            if verbose:
                print(f"  waves/SIMD cap {wv}: {t:.4f} ms", flush=True)
        best = min(table, key=lambda r: r[3])
        if len(ws) > 1:
            # the launch's tail: its last workgroups, ending at scattered
            # times, leave compute units idle; half-size chunks for the last
            # sweeps make those workgroups shorter
            for tl in TAIL_SWEEPS[1:]:
                t = run(best[0], sps, lpr, waves=best[4], block=best[5], best_of=rounds, tail=tl)
                table.append((best[0], sps, lpr, t, best[4], best[5], tl))
                if verbose:
                    print(f"  tail sweeps {tl}: {t:.4f} ms", flush=True)
            best = min(table, key=lambda r: r[3])
    rpl, sps, lpr, ms, waves, block, tail = best
    handle.set_tuning(kind, prec, runs_per_lane=rpl, steps_per_sync=sps, lanes_per_run=lpr,
                      waves_per_simd=waves, block=block, tail_sweeps=tail)
    return handle.get_tuning(kind, prec), ms, table


def tuned_handle(w, cache_path=None, device=0, **kw):
    """A handle tuned for ``w``: from the cache when it has the key, else by
    timing (and then stored in the cache)."""
    import torch
    h = cm.Handle(device)
    name = torch.cuda.get_device_name(device)
    key = cache_key(w, name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        t = cache[key]
        h.set_tuning(int(w["kind"]), int(w["precision"]), **t)
        return h, t, None
    t, ms, table = tune(h, w, **kw)
    if cache_path:
        cache[key] = t
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return h, t, table
