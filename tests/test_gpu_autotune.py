"""The autotuner on the device: it installs the shape it reports, the shape
leaves integer results unchanged, and the JSON cache is reused without
re-timing."""
import json

import numpy as np
import pytest

from paper_2110_15425_amd import autotune, cm, workloads as W

pytestmark = pytest.mark.gpu

CANDS = [(2, 8), (4, 16), (8, 4)]


def test_tune_installs_the_fastest_listed_shape():
    h = cm.Handle(0)
    w = W.conflict(trials=400, precision=W.FP32_STEP)
    before = cm.run(w, handle=h)
    t, ms, table = autotune.tune(h, w, reps=2, candidates=CANDS, finalists=2, rounds=2)
    assert all(len(r) == 7 for r in table)
    assert all(r[6] == 0 for r in table)  # one sweep: no tail axis
    shapes = table[:len(CANDS)]
    assert all(r[4:6] == (0, 256) for r in shapes)
    assert {(r[0], r[1]) for r in shapes} == set(CANDS)
    best = min(shapes, key=lambda r: r[3])
    # the workgroup-size axis on the best shape, with its runs per lane and half
    blocks = [r for r in table[len(CANDS):] if r[4] == 0]
    assert {r[5] for r in blocks} == {512, 1024}
    assert all(r[1] == best[1] and r[0] in (best[0], max(1, best[0] // 2)) for r in blocks)
    # the occupancy axis: the register caps timed on the best of those
    caps = [r for r in table if r[4] != 0]
    assert [r[4] for r in caps] == [4, 8]
    lead = min(shapes + blocks, key=lambda r: r[3])
    assert all((r[0], r[1], r[5]) == (lead[0], lead[1], lead[5]) for r in caps)
    fastest = min(table, key=lambda r: r[3])
    assert ms == fastest[3] > 0
    assert (t["runs_per_lane"], t["steps_per_sync"], t["waves_per_simd"], t["block"]) == \
        (fastest[0], fastest[1], fastest[4], fastest[5])
    assert h.get_tuning(W.LCA, W.FP32_STEP) == t
    after = cm.run(w, handle=h)
    for k in ("hist", "stats"):
        assert np.array_equal(before[k], after[k]), k


def test_tune_a_batch():
    h = cm.Handle(0)
    ws = [W.ddm(trials=5000, seed=s, precision=W.FP32_STEP) for s in (1, 2, 3)]
    t, ms, table = autotune.tune(h, ws, reps=2, candidates=[(2, 8), (4, 8, 64)], finalists=1,
                                 rounds=1)
    assert (t["runs_per_lane"], t["steps_per_sync"], t["lanes_per_run"]) in \
        {(2, 8, 1), (4, 8, 64)}
    assert ms > 0
    ws = [W.conflict(trials=2000, seed=s, grid=W.control_grid(4), precision=W.FP32_STEP) for s in (1, 2, 3)]
    t, ms, table = autotune.tune(h, ws, reps=2, candidates=[(2, 8)], finalists=1, rounds=1)
    tails = [r for r in table if r[6] != 0]  # a batch: the tail axis on the best shape
    assert [r[6] for r in tails] == [2, 4]
    assert t["tail_sweeps"] == min(table, key=lambda r: r[3])[6]


def test_tail_sweeps_leave_results_unchanged():
    """Half-size chunks for the last sweeps of a batched launch (and for
    cm_launch's one sweep) change only how runs are split among workgroups:
    every run's outcome, the histograms and the scores stay the same."""
    h = cm.Handle(0)
    ws = [W.conflict(trials=1500, seed=s, grid=W.control_grid(5), reward=1.0, cost=0.1,
                     precision=W.FP32_STEP) for s in (4, 5, 6)]
    ws.append(W.ddm(trials=3000, seed=7, drifts=np.linspace(0.0, 0.4, 3), precision=W.FP32_STEP))
    outs = []
    for tail in (0, 2, 12):
        h.set_tuning(W.LCA, W.FP32_STEP, tail_sweeps=tail, runs_per_lane=4)
        h.set_tuning(W.DDM, W.FP32_STEP, tail_sweeps=tail, lanes_per_run=1, runs_per_lane=3)
        assert h.get_tuning(W.LCA, W.FP32_STEP)["tail_sweeps"] == tail
        ds = [cm.DeviceSweep(h, w, dumps=True) for w in ws]
        cm.launch_batch(h, ds)
        outs.append([d.results() for d in ds] + [cm.run(ws[0], dumps=True, handle=h)])
    for o in outs[1:]:
        for i, (x, y) in enumerate(zip(outs[0], o)):
            for k in ("hist", "stats", "score", "best", "run_choice", "run_step", "run_flag", "run_state"):
                if x.get(k) is not None or y.get(k) is not None:
                    assert np.array_equal(x[k], y[k]), (i, k)
    for bad, st in ((dict(tail_sweeps=13), cm.E_INVALID),):
        with pytest.raises(cm.CmError) as e:
            h.set_tuning(W.LCA, W.FP32_STEP, **bad)
        assert e.value.status == st
    with pytest.raises(cm.CmError) as e:
        h.set_tuning(W.RNN, W.BF16_PROJ, tail_sweeps=2)
    assert e.value.status == cm.E_UNSUPPORTED


def test_tuned_handle_cache_round_trip(tmp_path):
    path = tmp_path / "tune.json"
    w = W.conflict(trials=300)
    h1, t1, table1 = autotune.tuned_handle(w, cache_path=str(path), reps=1, candidates=CANDS,
                                           finalists=1, rounds=1)
    assert table1 is not None  # timed
    cache = json.loads(path.read_text())
    assert list(cache.values()) == [t1]
    h2, t2, table2 = autotune.tuned_handle(w, cache_path=str(path), reps=1, candidates=CANDS)
    assert table2 is None  # from the cache
    assert t2 == t1
    assert h2.get_tuning(W.LCA, W.FP64) == t1


def test_fixed_knobs_are_refused_not_ignored():
    """The workgroup size and the rate-network tile are fixed; other values
    are refused as unsupported rather than accepted without effect."""
    h = cm.Handle(0)
    for bad in (dict(block=512), dict(tile_rows=32), dict(tile_rows=64)):
        with pytest.raises(cm.CmError) as e:
            h.set_tuning(W.RNN, W.BF16_PROJ, **bad)
        assert e.value.status == cm.E_UNSUPPORTED, bad
    h.set_tuning(W.RNN, W.BF16_PROJ, block=256, tile_rows=16)
    t = h.get_tuning(W.RNN, W.BF16_PROJ)
    assert (t["block"], t["tile_rows"]) == (256, 16)


@pytest.mark.parametrize("kind", ["lca", "ddm"])
def test_register_caps_leave_results_unchanged(kind):
    """The FP64 lane kernels built with registers capped for 4 or 8
    wavefronts per SIMD (the 8-wavefront build spills) compute exactly what
    the default build computes, per run, and match the oracle."""
    import oracle
    from parity import assert_parity
    h = cm.Handle(0)
    if kind == "lca":
        w = W.conflict(trials=700, grid=W.control_grid(6), reward=1.0, cost=0.1, seed=21)
        k = W.LCA
    else:
        w = W.ddm(trials=4000, drifts=np.linspace(-0.3, 0.5, 5), seed=22)
        k = W.DDM
    outs = []
    for wv in (0, 4, 8):
        h.set_tuning(k, W.FP64, waves_per_simd=wv, lanes_per_run=1 if kind == "ddm" else 0)
        assert h.get_tuning(k, W.FP64)["waves_per_simd"] == wv
        outs.append(cm.run(w, dumps=True, handle=h))
    for o in outs[1:]:
        for key in ("hist", "stats", "run_choice", "run_step", "run_flag", "run_state"):
            assert np.array_equal(outs[0][key], o[key]), key
    orc = oracle.run(w, dumps=True)
    correct = [1]
    if kind == "lca":
        correct = oracle.conflict_correct(w["weights"], w["params"][W.LCA_P["hid_gain"]],
                                          w["params"][W.LCA_P["hid_bias"]])
    assert_parity(w, outs[2], orc, correct)


@pytest.mark.parametrize("kind,prec", [("lca", W.FP64), ("lca", W.FP32_STEP), ("ddm", W.FP64)])
def test_workgroup_sizes_leave_results_unchanged(kind, prec):
    """Lane kernels in workgroups of 512 and 1024 threads (one drain packing
    over more wavefronts; several sweeps in one launch) compute per run
    exactly what 256-thread workgroups compute, and match the oracle (FP64)."""
    import oracle
    from parity import assert_parity
    h = cm.Handle(0)
    if kind == "lca":
        ws = [W.conflict(trials=900, grid=W.control_grid(6)[::3], reward=1.0, cost=0.1, seed=s,
                         precision=prec) for s in (31, 32)]
        k = W.LCA
    else:
        ws = [W.ddm(trials=3000, drifts=np.linspace(-0.3, 0.5, 5), seed=s) for s in (33, 34)]
        k = W.DDM
    outs = []
    for blk in (256, 512, 1024):
        h.set_tuning(k, prec, block=blk, runs_per_lane=3, lanes_per_run=1 if kind == "ddm" else 0)
        assert h.get_tuning(k, prec)["block"] == blk
        outs.append([cm.run(w, dumps=True, handle=h) for w in ws])
        ds = [cm.DeviceSweep(h, w) for w in ws]
        cm.launch_batch(h, ds)
        outs[-1].append([d.results() for d in ds])
    for o in outs[1:]:
        for i in range(2):
            for key in ("hist", "stats", "run_choice", "run_step", "run_flag", "run_state"):
                assert np.array_equal(outs[0][i][key], o[i][key]), (i, key)
            for key in ("hist", "stats"):
                assert np.array_equal(outs[0][i][key], o[2][i][key]), ("batch", i, key)
    if prec == W.FP64:
        correct = [1]
        if kind == "lca":
            correct = oracle.conflict_correct(ws[0]["weights"], ws[0]["params"][W.LCA_P["hid_gain"]],
                                              ws[0]["params"][W.LCA_P["hid_bias"]])
        assert_parity(ws[0], outs[2][0], oracle.run(ws[0], dumps=True), correct)


def test_workgroup_size_rejected_where_not_built():
    h = cm.Handle(0)
    for k, p in ((W.LCA, W.FP64), (W.RNN, W.BF16_PROJ)):
        with pytest.raises(cm.CmError) as e:
            h.set_tuning(k, p, block=768 if k == W.LCA else 512)
        assert e.value.status == cm.E_UNSUPPORTED


def test_register_cap_rejected_where_not_built():
    h = cm.Handle(0)
    with pytest.raises(cm.CmError) as e:
        h.set_tuning(W.LCA, W.FP64, waves_per_simd=6)
    assert e.value.status == cm.E_UNSUPPORTED
    with pytest.raises(cm.CmError) as e:
        h.set_tuning(W.RNN, W.BF16_PROJ, waves_per_simd=4)
    assert e.value.status == cm.E_UNSUPPORTED
