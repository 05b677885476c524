"""cm_launch_graph: the batched launch replayed from the handle's graph cache.

Every replay must equal the eager cm_launch_batch of the same sweeps: with
eager work of the program's own between replays, with the outputs
overwritten between replays (the graph's preparation kernels re-zero them),
after an argument change (a new capture), and after more argument sets than
the cache keeps (the least recently used is dropped and captured again)."""
import numpy as np
import pytest
import torch

from paper_2110_15425_amd import cm, workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("hist", "stats", "score", "best", "run_choice", "run_step", "run_flag", "run_state")


def _mix(seed=0):
    return [W.conflict(trials=700, seed=3 + seed, grid=W.control_grid(4), precision=W.FP32_STEP),
            W.conflict(trials=500, seed=4 + seed, grid=W.control_grid(3), reward=1.0, cost=0.1),
            W.ddm(trials=3000, seed=5 + seed, drifts=np.linspace(0.0, 0.5, 4)),
            W.rnn(trials=64, n_units=64, seed=6 + seed),
            W.control_loop(trials=40, seed=7 + seed, levels=3, samples=2)]


def _results(ds):
    return [d.results() for d in ds]


def _same(a, b, what):
    for i, (x, y) in enumerate(zip(a, b)):
        for k in KEYS:
            if k in x or k in y:
                assert np.array_equal(x[k], y[k]), (what, i, k)


def _scribble(ds):
    for d in ds:
        for name in ("hist", "stats", "score", "best", "run_choice", "run_step", "run_flag", "run_state"):
            t = getattr(d, name, None)
            if t is not None:
                t.fill_(7)


def test_graph_replays_equal_the_eager_batch():
    h = cm.Handle(0)
    ws = _mix()
    ref_ds = [cm.DeviceSweep(h, w, dumps=True) for w in ws]
    cm.launch_batch(h, ref_ds)
    ref = _results(ref_ds)
    ds = [cm.DeviceSweep(h, w, dumps=True) for w in ws]
    other = W.conflict(trials=300, seed=99, grid=W.control_grid(2))
    for rep in range(4):
        print(f"graph replay {rep}", flush=True)
        cm.launch_graph(h, ds)
        torch.cuda.synchronize()
        _same(_results(ds), ref, f"replay {rep}")
        _scribble(ds)  # the next replay must re-zero every output
        cm.run(other, handle=h)  # eager work of the program's own between replays
        torch.cuda.synchronize()


def test_graph_recaptures_on_a_changed_argument():
    h = cm.Handle(0)
    ws = _mix()
    ds = [cm.DeviceSweep(h, w) for w in ws]
    cm.launch_graph(h, ds)
    torch.cuda.synchronize()
    first = _results(ds)
    # a new seed in one sweep: a different argument set, so a new graph
    ws2 = list(ws)
    ws2[0] = W.with_(ws[0], seed=123)
    ds2 = [cm.DeviceSweep(h, w) for w in ws2]
    ref2 = [cm.DeviceSweep(h, w) for w in ws2]
    cm.launch_batch(h, ref2)
    cm.launch_graph(h, ds2)
    torch.cuda.synchronize()
    _same(_results(ds2), _results(ref2), "changed seed")
    assert not np.array_equal(_results(ds2)[0]["hist"], first[0]["hist"])
    # the first argument set replays its own graph, unchanged
    _scribble(ds)
    cm.launch_graph(h, ds)
    torch.cuda.synchronize()
    _same(_results(ds), first, "first set again")


def test_graph_cache_eviction_and_clear():
    h = cm.Handle(0)
    w = W.conflict(trials=200, grid=W.control_grid(2), precision=W.FP32_STEP)
    sets = [[cm.DeviceSweep(h, W.with_(w, seed=s))] for s in range(1, 20)]  # more than the cache keeps
    refs = []
    for ds in sets:
        r = [cm.DeviceSweep(h, ds[0].w)]
        cm.launch_batch(h, r)
        refs.append(_results(r))
    for rnd in range(2):  # the second round finds the first sets evicted and captures them again
        for ds, ref in zip(sets, refs):
            _scribble(ds)
            cm.launch_graph(h, ds)
        torch.cuda.synchronize()
        for i, (ds, ref) in enumerate(zip(sets, refs)):
            _same(_results(ds), ref, f"round {rnd} set {i}")
    cm.graph_clear(h)
    _scribble(sets[0])
    cm.launch_graph(h, sets[0])
    torch.cuda.synchronize()
    _same(_results(sets[0]), refs[0], "after clear")


def test_graph_launch_rejects_what_the_batch_rejects():
    h = cm.Handle(0)
    good = cm.DeviceSweep(h, W.ddm(trials=100))
    bad = cm.DeviceSweep(h, W.ddm(trials=100))
    bad.sweep.n_bins = 0
    with pytest.raises(cm.CmError) as e:
        cm.launch_graph(h, [good, bad])
    assert e.value.status == cm.E_INVALID
