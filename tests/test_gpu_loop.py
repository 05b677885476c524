"""Closed-loop control on the GPU against the oracle: per-run choice and
decision step bit-exact on unflagged runs (FP64), and a one-allocation loop
identical to the open-loop LCA kernel in both precisions."""
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import cm, workloads as W
from parity import assert_parity, hist_l1

pytestmark = pytest.mark.gpu

CASES = {
    # team of 1 lane: one allocation
    "one_allocation": W.control_loop(trials=450, levels=1, amax=1.3, samples=2, costs=[0.0, 0.2]),
    # team of 4 lanes, all busy
    "levels2": W.control_loop(trials=360, levels=2, samples=3, costs=[0.0, 0.01]),
    # team of 16 lanes, 9 busy
    "levels3_ragged": W.control_loop(trials=301, levels=3, samples=1, costs=[0.0, 0.05, 0.3],
                                     seed=5),
    # team of 64 lanes, exactly one allocation each
    "levels8": W.control_loop(trials=450, levels=8, samples=4, costs=[0.0, 0.003, 0.01, 0.3]),
    # more allocations than lanes: lanes stride
    "levels10_stride": W.control_loop(trials=180, levels=10, samples=2, costs=[0.01], seed=7),
    # wide searches: each lane evaluates four allocations at a time, the last
    # group ragged (289 = 4 x 64 + 33) or whole (1024 = 4 groups of 4 x 64)
    "levels17_chains": W.control_loop(trials=120, levels=17, samples=2, costs=[0.0, 0.02],
                                      seed=8),
    # 1024 allocations: few runs take a whole workgroup per run (four
    # wavefronts folding through LDS), many runs a wavefront each
    "levels32_workgroup": W.control_loop(trials=60, levels=32, samples=1, costs=[0.003], seed=9),
    "levels32_wavefront": W.control_loop(trials=4100, levels=32, samples=1, costs=[0.0, 0.003],
                                         seed=10, max_steps=60, n_bins=6),
    "no_signals_short_cap": W.control_loop(trials=200, levels=5, samples=2, max_steps=15,
                                           n_bins=5),
    "nonneg": W.control_loop(trials=180, levels=4, samples=2, nonneg=1.0, costs=[0.0, 0.01]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_loop_fp64_parity(name):
    w = CASES[name]
    print(f"case {name} S={w['n_settings']} T={w['trials']}", flush=True)
    g = cm.run(w, dumps=True)
    o = oracle.run(w, dumps=True)
    correct = oracle.conflict_correct(w["weights"], w["params"][W.LOOP_P["hid_gain"]],
                                      w["params"][W.LOOP_P["hid_bias"]])
    assert_parity(w, g, o, correct)


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_STEP])
def test_one_allocation_loop_equals_open_loop_kernel(prec):
    loop = W.control_loop(trials=2000, levels=1, amax=0.7, samples=3, costs=[0.0, 1.0],
                          precision=prec)
    lca = W.conflict(trials=2000, grid=np.array([[0.7, 0.7], [0.7, 0.7]]), precision=prec)
    a, b = cm.run(loop, dumps=True), cm.run(lca, dumps=True)
    for k in ("run_choice", "run_step", "run_state", "hist"):
        assert np.array_equal(a[k], b[k]), k


def test_loop_fp32_against_fp64_oracle():
    w = W.control_loop(trials=900, levels=6, samples=3, costs=[0.0, 0.01, 0.3],
                       precision=W.FP32_STEP)
    g = cm.run(w)
    o = oracle.run(W.with_(w, precision=W.FP64))
    l1 = hist_l1(g, o, int(w["trials"]))
    print("fp32 loop histogram L1 per setting", l1)
    # paired streams: FP32 follows FP64 closely, but a flipped allocation
    # choice decorrelates the rest of a run, so allow sampling-size changes
    assert np.all(l1 < 0.25)
    pc_g = g["stats"][:, 3] / w["trials"]
    pc_o = o["stats"][:, 3] / w["trials"]
    assert np.all(np.abs(pc_g - pc_o) < 0.05), (pc_g, pc_o)
