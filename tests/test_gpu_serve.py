"""Serving on the GPU: every request's outputs are the same alone and when
served in a concurrent mix."""
import numpy as np
import pytest

from paper_2110_15425_amd import cm, serve

pytestmark = pytest.mark.gpu


def test_mix_equals_alone():
    h = cm.Handle(0)
    mix = serve.served_mix(24, rate_hz=1e6, seed=5, max_runs=20_000)  # all arrive at once
    done = serve.run_mix(h, mix, budget_bytes=4 << 30, n_streams=4)
    assert len(done) == 24
    for r in done:
        alone = cm.run(r.w, handle=h)
        for k in ("hist", "stats", "score", "best"):
            if alone[k] is None:
                continue
            assert np.array_equal(r.result[k], alone[k]), (r.rid, k)
    lat = serve.latency_summary(done)
    print(lat)
    assert lat["p99_ms"] >= lat["p50_ms"] > 0


def test_mix_through_the_device_queue_equals_alone():
    """The same served mix with the conflict-network FP32 requests going
    through the device work queue (one persistent kernel) and the rest
    through the slots: every request's outputs equal its lone launch."""
    h = cm.Handle(0)
    mix = serve.served_mix(24, rate_hz=1e6, seed=5, max_runs=20_000)
    done = serve.run_mix(h, mix, budget_bytes=4 << 30, n_streams=4, queue=True)
    assert len(done) == 24
    for r in done:
        alone = cm.run(r.w, handle=h)
        for k in ("hist", "stats", "score", "best"):
            if alone[k] is None:
                continue
            assert np.array_equal(r.result[k], alone[k]), (r.rid, k)
    print(serve.latency_summary(done))


def test_budget_smaller_than_mix_still_completes():
    h = cm.Handle(0)
    mix = serve.served_mix(16, rate_hz=1e6, seed=6, max_runs=10_000)
    biggest = max(serve.request_bytes(w) for _, w in mix)
    done = serve.run_mix(h, mix, budget_bytes=biggest + 1, n_streams=2)
    assert len(done) == 16


def test_submit_poll_matches_launch():
    """cm_submit / cm_poll: the host copies it enqueues hold the same results as
    a plain launch, for a mixed batch of kinds on several slots."""
    from paper_2110_15425_amd import workloads as W
    h = cm.Handle(0)
    cm.serve_config(h, 3)
    groups = [[W.ddm(trials=3000, seed=3), W.conflict(trials=200, seed=4, precision=W.FP32_STEP)],
              [W.grid_search(trials=20, seed=5)],
              [W.rnn(trials=256, seed=6, precision=W.BF16_PROJ), W.ddm(trials=500, seed=7)]]
    tickets = []
    for ws in groups:
        ds = [cm.DeviceSweep(h, w) for w in ws]
        host = [cm.host_buffers(d) for d in ds]
        t = cm.submit(h, ds, host)
        assert t is not None and t > 0
        tickets.append((t, ws, ds, host))
    import time
    t0 = time.time()
    pending = list(tickets)
    while pending:
        pending = [x for x in pending if not cm.poll(h, x[0])]
        assert time.time() - t0 < 60
    for t, ws, ds, host in tickets:
        assert cm.poll(h, t)  # stays done
        for w, hh in zip(ws, host):
            alone = cm.run(w, handle=h)
            for k, v in hh.items():
                got = v.numpy().view(np.uint64) if k in ("hist", "stats") else v.numpy()
                assert np.array_equal(got, alone[k]), (k, int(w["kind"]))


def test_submit_reports_busy_slots():
    """With one slot held by unfinished work, a second submit is refused with
    CM_E_BUSY (nothing enqueued) and succeeds once the first is done."""
    import time
    import torch
    from paper_2110_15425_amd import workloads as W
    h = cm.Handle(0)
    cm.serve_config(h, 1)
    d1 = cm.DeviceSweep(h, W.ddm(trials=2000, seed=1))
    d2 = cm.DeviceSweep(h, W.ddm(trials=2000, seed=2))
    producer = torch.cuda.Stream()
    with torch.cuda.stream(producer):
        torch.cuda._sleep(200_000_000)  # keeps the producer, and so the slot, busy
    t1 = cm.submit(h, [d1], producer=producer)
    assert t1 is not None
    assert cm.submit(h, [d2]) is None
    assert not cm.poll(h, t1)
    t0 = time.time()
    while not cm.poll(h, t1):
        assert time.time() - t0 < 60
    t2 = cm.submit(h, [d2])
    assert t2 is not None and t2 > t1
    while not cm.poll(h, t2):
        assert time.time() - t0 < 60
    for d, seed in ((d1, 1), (d2, 2)):
        alone = cm.run(W.ddm(trials=2000, seed=seed), handle=h)
        assert np.array_equal(d.results()["hist"], alone["hist"])
    with pytest.raises(cm.CmError):
        cm.poll(h, t2 + 100)


def _correct(w):
    import oracle
    from paper_2110_15425_amd import workloads as W
    if w["kind"] == W.DDM:
        return [1]
    if w["kind"] == W.LCA:
        return oracle.conflict_correct(w["weights"], w["params"][W.LCA_P["hid_gain"]],
                                       w["params"][W.LCA_P["hid_bias"]])
    return [-1]


def test_fp64_mix_matches_oracle():
    """An FP64 served mix of all four configurations (16 requests arriving
    together, overlapping on four slots, grouped into batched launches)
    against the FP64 oracle: every request's per-run choice and decision
    step bit-exact on unflagged runs, final states within the FP64
    tolerance, and the served histograms, statistics, scores and best
    setting equal to the oracle's (after removing flagged runs, if any)."""
    import oracle
    from parity import assert_parity
    h = cm.Handle(0)
    mix = serve.served_mix(16, rate_hz=1e6, seed=8, max_runs=3000, fp32=False)
    kinds = sorted({(int(w["kind"]), float(w["reward"])) for _, w in mix})
    assert len(kinds) == 4, kinds  # DDM, conflict LCA, scored grid, rate network
    done = serve.run_mix(h, mix, budget_bytes=4 << 30, n_streams=4, dumps=True)
    assert len(done) == 16
    for r in sorted(done, key=lambda r: r.rid):
        w = r.w
        print(f"case served request {r.rid} kind={w['kind']} S={w['n_settings']} "
              f"T={w['trials']}", flush=True)
        g = dict(r.result)
        d = g.pop("device_sweep").results()
        for k in ("run_choice", "run_step", "run_flag", "run_state"):
            g[k] = d[k]
        for k in ("hist", "stats", "score", "best"):  # the host copies are the device's
            if d[k] is not None:
                assert np.array_equal(g[k], d[k]), k
        o = oracle.run(w, dumps=True)
        assert_parity(w, g, o, _correct(w))
        if o["score"] is not None:
            flagged = (g["run_flag"] != 0) | (o["run_flag"] != 0)
            if not flagged.any():
                assert np.array_equal(g["score"], o["score"])
                assert np.array_equal(g["best"], o["best"])
