"""Coarse-to-fine control search by simulation.

The Distill paper narrows a control space by repeatedly bisecting it, keeping
the region with the better outcome, until the optimum is located after a few
rounds instead of hundreds of thousands of runs (Sec. 4.3, where the ranges
come from value-range analysis).  Here the ranges come from simulation: each
round evaluates an n x n grid of control allocations over the current box on
the GPU (one scored sweep), keeps the best allocation, and shrinks the box to
one grid cell around it.  Every round is one libcm sweep; the search itself
is a few lines of host logic.
"""
import numpy as np

from . import cm, workloads as W


def refine(handle, make_workload, lo=(0.0, 0.0), hi=(5.0, 5.0), n=8, rounds=4, seed=1):
    """Run the search.  ``make_workload(grid, seed)`` builds a scored sweep over
    the [settings x 2] grid.  Returns a list of per-round dicts (box, best
    allocation, best score, runs used) and the final best allocation."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    history = []
    best_c = None
    for r in range(rounds):
        grid = box_grid(lo, hi, n)
        w = make_workload(grid, seed + r)
        out = cm.run(w, handle=handle)
        s = int(out["best"][0])
        best_c = grid[s].copy()
        history.append(dict(round=r, lo=lo.tolist(), hi=hi.tolist(), best=best_c.tolist(),
                            best_index=s, score=float(out["score"][s]), ties=int(out["best"][1]),
                            scores=out["score"].copy(), seed=seed + r,
                            runs=int(w["n_settings"] * w["trials"])))
        lo, hi = narrow(lo, hi, n, best_c)
    return history, best_c


def box_grid(lo, hi, n):
    """The n x n grid of allocations over the box [lo, hi] (row-major in the
    first signal), as [n*n x 2]."""
    a = np.linspace(lo[0], hi[0], n)
    b = np.linspace(lo[1], hi[1], n)
    A, B = np.meshgrid(a, b, indexing="ij")
    return np.stack([A.ravel(), B.ravel()], 1)


def narrow(lo, hi, n, best_c):
    """The next round's box: one grid cell around the best allocation,
    clipped to the current box."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    step = (hi - lo) / (n - 1)
    return np.maximum(lo, best_c - step), np.minimum(hi, best_c + step)


def conflict_search(trials=400, precision=W.FP32_STEP):
    """The conflict-network control search (reward 1, cost 0.1)."""
    def make(grid, seed):
        return W.conflict(trials=trials, seed=seed, grid=grid, reward=1.0, cost=0.1,
                          precision=precision)
    return make
