"""Batching and graph capture: several sweeps in one call give exactly the
results of separate calls; a captured HIP graph replays to the eager
results every time."""
import numpy as np
import pytest

from paper_2110_15425_amd import cm, workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("hist", "stats", "score", "best")


def _same(a, b):
    for k in KEYS:
        if a[k] is None:
            assert b[k] is None
        else:
            assert np.array_equal(a[k], b[k]), k


def _mix():
    return [
        W.ddm(trials=3000, seed=2),
        W.ddm(trials=700, seed=3, drifts=np.linspace(0, 0.6, 9), precision=W.FP32_STEP),
        W.conflict(trials=900, seed=4, grid=W.control_grid(3)),
        W.grid_search(n=10, trials=50, seed=5),
        W.conflict(trials=5, seed=6, grid=W.control_grid(30)),
        W.conflict(trials=2000, seed=7, precision=W.FP32_STEP),
        W.rnn(trials=300, seed=8, n_units=64, weights=W.rnn_weights(64, 7),
              precision=W.BF16_PROJ),
        W.ddm(trials=1, seed=9),
    ]


def test_batch_equals_separate_launches():
    h = cm.Handle(0)
    ws = _mix()
    alone = [cm.run(w, handle=h) for w in ws]
    ds = [cm.DeviceSweep(h, w) for w in ws]
    cm.launch_batch(h, ds)
    for d, a in zip(ds, alone):
        _same(d.results(), a)


def test_batch_larger_than_one_launch():
    h = cm.Handle(0)
    ws = [W.conflict(trials=100 + 37 * i, seed=20 + i, grid=W.control_grid(2)) for i in range(27)]
    alone = [cm.run(w, handle=h) for w in ws]
    ds = [cm.DeviceSweep(h, w) for w in ws]
    cm.launch_batch(h, ds)
    for d, a in zip(ds, alone):
        _same(d.results(), a)


@pytest.mark.parametrize("rpl,sps", [(6, 12), (8, 16)])
def test_benchmark_batched_launch(rpl, sps):
    """The benchmark's timed launch: twelve C1 sweeps (noise seeds 1..12) in
    FP32 steps as one batched launch at a shape the autotuner picks there;
    each sweep's integers equal the same sweep launched alone at the default
    shape, and the first is within the FP32 accuracy bound of the FP64
    oracle on its paired streams."""
    import oracle
    from parity import hist_l1

    w32 = W.with_(W.conflict(reward=1.0, cost=0.1), precision=W.FP32_STEP)
    ws = [W.with_(w32, seed=1 + i) for i in range(12)]
    print(f"case benchmark batch x12 rpl={rpl} sps={sps}", flush=True)
    h = cm.Handle(0)
    h.set_tuning(W.LCA, W.FP32_STEP, runs_per_lane=rpl, steps_per_sync=sps)
    ds = [cm.DeviceSweep(h, w) for w in ws]
    cm.launch_batch(h, ds)
    got = [d.results() for d in ds]
    h0 = cm.Handle(0)
    for w, g in zip(ws, got):
        _same(g, cm.run(w, handle=h0))
    o64 = oracle.run(W.with_(ws[0], precision=W.FP64))
    assert hist_l1(got[0], o64, int(w32["trials"])).max() < 0.02


def test_batch_rejects_whole_batch_on_one_bad_entry():
    h = cm.Handle(0)
    good = cm.DeviceSweep(h, W.ddm(trials=10))
    bad = cm.DeviceSweep(h, W.ddm(trials=10))
    bad.sweep.n_bins = 0
    with pytest.raises(cm.CmError) as e:
        cm.launch_batch(h, [good, bad])
    assert "batch entry 1" in str(e.value)


def test_graph_replay_matches_eager():
    import torch
    h = cm.Handle(0)
    w = W.grid_search(n=16, trials=64, seed=11)
    eager = cm.run(w, handle=h)
    ds = cm.DeviceSweep(h, w)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture
        ds.launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ds.launch()
    for rep in range(4):
        # eager work on the device between replays
        other = cm.run(W.ddm(trials=500, seed=rep), handle=h)
        assert other["stats"][0, :3].sum() == 500
        ds.hist.fill_(-1)
        ds.stats.fill_(-1)
        g.replay()
        _same(ds.results(), eager)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["ddm", "lca"])
def test_unfused_equals_fused(kind, prec):
    """The node-by-node execution computes exactly what the fused kernels do."""
    p = W.FP64 if prec == "fp64" else W.FP32_STEP
    w = (W.ddm(trials=3000, seed=3, drifts=np.linspace(0, 0.6, 5), precision=p) if kind == "ddm"
         else W.grid_search(n=6, trials=300, seed=4, precision=p))
    h = cm.Handle(0)
    fused = cm.run(w, dumps=True, handle=h)
    ds = cm.DeviceSweep(h, w, dumps=True)
    ds.launch_unfused()
    got = ds.results()
    for k in ("hist", "stats", "score", "best", "run_choice", "run_step", "run_flag"):
        if fused.get(k) is not None:
            assert np.array_equal(got[k], fused[k]), k
    # identical arithmetic: even the final states agree bit for bit (lane-per-run DDM/LCA)
    if kind == "lca":
        assert np.array_equal(got["run_state"], fused["run_state"])


def _correct(w):
    import oracle
    if w["kind"] == W.DDM:
        return [1]
    return oracle.conflict_correct(w["weights"], w["params"][W.LCA_P["hid_gain"]],
                                   w["params"][W.LCA_P["hid_bias"]])


UNFUSED_ORACLE_CASES = {
    "ddm_drifts_ragged": lambda: W.ddm(trials=3001, seed=3, drifts=np.linspace(0, 0.6, 5)),
    "ddm_short_cap": lambda: W.ddm(trials=900, seed=8, max_steps=77, n_bins=7, noise=0.3),
    "lca_grid_scored": lambda: W.grid_search(n=6, trials=301, seed=4),
    "lca_nonneg": lambda: W.conflict(trials=700, seed=7, nonneg=1.0, max_steps=300, n_bins=30,
                                     grid=W.control_grid(3)),
    "c1_full": lambda: W.conflict(),
}


@pytest.mark.parametrize("name", list(UNFUSED_ORACLE_CASES))
def test_unfused_fp64_against_oracle(name):
    """The node-by-node kernels (their own arithmetic, state through HBM
    every step) against the FP64 oracle: per-run integers bit-exact on
    unflagged runs, final states within the FP64 tolerance, histograms,
    statistics, scores and best setting equal."""
    import oracle
    from parity import assert_parity
    w = UNFUSED_ORACLE_CASES[name]()
    print(f"case unfused {name} kind={w['kind']} S={w['n_settings']} T={w['trials']}", flush=True)
    h = cm.Handle(0)
    ds = cm.DeviceSweep(h, w, dumps=True)
    ds.launch_unfused()
    g = ds.results()
    o = oracle.run(w, dumps=True)
    assert_parity(w, g, o, _correct(w))
    if o["score"] is not None and not ((g["run_flag"] != 0) | (o["run_flag"] != 0)).any():
        assert np.array_equal(g["score"], o["score"])
        assert np.array_equal(g["best"], o["best"])


def test_refine_fp64_against_oracle():
    """The coarse-to-fine search in FP64 against the oracle, round by round:
    each round's score surface and best allocation equal the oracle's on the
    same grid and seed, and each next box is the one the oracle's best
    allocation gives, so the whole search is the oracle's search."""
    import oracle
    from paper_2110_15425_amd import refine
    h = cm.Handle(0)
    n, rounds = 5, 3
    make = refine.conflict_search(trials=300, precision=W.FP64)
    hist, best = refine.refine(h, make, n=n, rounds=rounds)
    lo, hi = np.zeros(2), np.full(2, 5.0)
    for r in hist:
        print(f"case refine round {r['round']} box {r['lo']} {r['hi']}", flush=True)
        assert np.allclose(r["lo"], lo, rtol=0, atol=0) and np.allclose(r["hi"], hi, rtol=0, atol=0)
        grid = refine.box_grid(lo, hi, n)
        o = oracle.run(make(grid, r["seed"]))
        assert int(o["stats"][:, 8].sum()) == 0, "flagged runs in a refinement round"
        assert np.array_equal(r["scores"], o["score"])
        assert r["best_index"] == int(o["best"][0]) and r["ties"] == int(o["best"][1])
        lo, hi = refine.narrow(lo, hi, n, grid[int(o["best"][0])])
    assert np.array_equal(best, refine.box_grid(hist[-1]["lo"], hist[-1]["hi"], n)[hist[-1]["best_index"]])


def test_coarse_to_fine_search_matches_full_grid():
    """Four rounds of a 6x6 grid (57,600 runs) find an allocation as good as
    the best of the exhaustive 64x64 grid (409,600 runs), judged by a
    separate high-trial evaluation of both."""
    from paper_2110_15425_amd import refine
    h = cm.Handle(0)
    hist, best = refine.refine(h, refine.conflict_search(trials=400), n=6, rounds=4)
    assert sum(r["runs"] for r in hist) == 4 * 36 * 400
    full = cm.run(W.grid_search(precision=W.FP32_STEP), handle=h)
    gbest = W.control_grid(64)[int(full["best"][0])]
    evalw = W.conflict(trials=40_000, seed=99, grid=np.stack([best, gbest]), reward=1.0, cost=0.1,
                       precision=W.FP32_STEP)
    sc = cm.run(evalw, handle=h)["score"]
    print("refined", best, sc[0], "full grid", gbest, sc[1], [r["score"] for r in hist])
    assert sc[0] >= sc[1] - 0.02


def _capture(fn):
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


@pytest.mark.parametrize("what", ["batch", "timecourse", "loop", "rate_network"])
def test_graph_replays_of_every_launch_kind(what):
    """A captured launch (batched sweeps of two kinds, the time course, the
    closed loop, the rate network) replayed several times, with other eager
    work between replays, gives the eager result every time: the library's
    preparation kernel clears the outputs inside the graph (no memset nodes)."""
    h = cm.Handle(0)
    if what == "batch":
        ws = [W.ddm(trials=700, seed=2, drifts=[0.1, 0.4]), W.grid_search(n=5, trials=40, seed=3),
              W.ddm(trials=300, seed=4, precision=W.FP32_STEP)]
        ds = [cm.DeviceSweep(h, w) for w in ws]
        eager = [cm.run(w, handle=h) for w in ws]
        g = _capture(lambda: cm.launch_batch(h, ds))
    elif what == "timecourse":
        w = W.conflict(trials=300, grid=W.control_grid(3), precision=W.FP32_STEP)
        ds = [cm.DeviceSweep(h, w)]
        eager_out, eager_tc = cm.timecourse(w, 7, handle=h)
        eager = [eager_out]
        # the output tensor allocated during capture comes from the graph's pool
        g = _capture(lambda: ds[0].launch_timecourse(7))
        tc_buf = ds[0].timecourse
    elif what == "loop":
        w = W.control_loop(trials=200, levels=4, samples=2, costs=[0.0, 0.02])
        ds = [cm.DeviceSweep(h, w)]
        eager = [cm.run(w, handle=h)]
        g = _capture(ds[0].launch)
    else:
        w = W.rnn(trials=512, n_units=64, precision=W.BF16_PROJ)
        ds = [cm.DeviceSweep(h, w)]
        eager = [cm.run(w, handle=h)]
        g = _capture(ds[0].launch)
    for rep in range(3):
        other = cm.run(W.ddm(trials=500, seed=10 + rep), handle=h)
        assert other["stats"][0, :3].sum() == 500
        for d in ds:
            d.hist.fill_(-1)
            d.stats.fill_(-1)
        if what == "timecourse":
            tc_buf.fill_(-1)
        g.replay()
        for d, e in zip(ds, eager):
            _same(d.results(), e)
        if what == "timecourse":
            assert np.array_equal(tc_buf.cpu().numpy(), eager_tc)


@pytest.mark.parametrize("kind", ["ddm", "lca"])
@pytest.mark.parametrize("prec", [W.FP64, W.FP32_STEP])
def test_measured_ceiling_bounds_the_sweeps(kind, prec):
    """The ceiling kernel (the step's random numbers and update alone) runs
    faster per run-step than a whole sweep of the same model and precision."""
    import time
    import torch
    h = cm.Handle(0)
    w = W.ddm(trials=2_000_000, precision=prec) if kind == "ddm" else \
        W.conflict(precision=prec)
    c = cm.ceiling(w, handle=h)
    ds = cm.DeviceSweep(h, w)
    ds.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ds.launch()
    torch.cuda.synchronize()
    rate = cm.run_steps(w, ds.results()) / (time.perf_counter() - t0)
    print(f"{kind} prec {prec}: ceiling {c:.3e}, sweep {rate:.3e} run-steps/s")
    assert c > rate > 0


def test_ddm_form_independent_of_batch_partners():
    """A small DDM sweep (wavefront-scan form) batched with one of more than
    2^20 runs (lane form) computes bit for bit what it computes alone: the
    batch launches each form separately."""
    h = cm.Handle(0)
    small = W.ddm(trials=3000, seed=2)
    big = W.ddm(trials=(1 << 20) + 5, seed=3, max_steps=200, n_bins=10)
    print("case ddm small + 2^20+5 batch", flush=True)
    alone = cm.run(small, dumps=True, handle=h)
    ds = [cm.DeviceSweep(h, small, dumps=True), cm.DeviceSweep(h, big)]
    cm.launch_batch(h, ds)
    got = ds[0].results()
    for k in ("run_state", "run_choice", "run_step", "run_flag", "hist", "stats"):
        assert np.array_equal(got[k], alone[k]), k
    big_alone = cm.run(big, handle=h)
    _same(ds[1].results(), big_alone)
