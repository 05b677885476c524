"""Device work queue (cm_queue_*): one persistent kernel fed with requests.

Every request's outputs must equal cm_launch's for the same sweep (integer
outputs and dumps bit for bit; the FP64 form also matches the oracle),
whether requests are submitted together, one after another while earlier
ones run, or after the kernel has gone idle and ended; a full queue refuses
new work instead of overwriting it."""
import time

import numpy as np
import pytest

from paper_2110_15425_amd import cm, workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("hist", "stats", "score", "best", "run_choice", "run_step", "run_flag", "run_state")


def _wait(q, tickets, limit_s=60.0):
    left = set(tickets)
    t0 = time.time()
    while left:
        for t in list(left):
            if q.poll(t):
                left.discard(t)
        assert time.time() - t0 < limit_s, f"requests {sorted(left)} not done after {limit_s} s"
        time.sleep(0.0005)


def _same(x, y, what):
    for k in KEYS:
        if k in x or k in y:
            assert np.array_equal(x[k], y[k]), (what, k)


def _requests(prec):
    g = W.control_grid(8)
    return [W.conflict(trials=700, seed=11, grid=g[::7], precision=prec),
            W.conflict(trials=90, seed=12, grid=g, reward=1.0, cost=0.1, precision=prec),
            W.conflict(trials=3000, seed=13, grid=g[:3], precision=prec),
            W.conflict(trials=1, seed=14, grid=g[:5], precision=prec)]


@pytest.mark.parametrize("prec", [W.FP32_STEP, W.FP64])
def test_queue_results_equal_launch(prec):
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, prec, slots=8, idle_us=20000)
    try:
        ws = _requests(prec)
        ds = [cm.DeviceSweep(h, w, dumps=True) for w in ws]
        print(f"queue prec={prec}: submitting {len(ds)} requests", flush=True)
        tickets = [q.submit(d) for d in ds]
        _wait(q, tickets)
        for i, (w, d) in enumerate(zip(ws, ds)):
            _same(d.results(), cm.run(w, dumps=True, handle=h), f"request {i}")
    finally:
        q.close()


def test_queue_fp64_matches_oracle():
    import oracle
    from parity import assert_parity
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, W.FP64, slots=2, idle_us=20000)
    try:
        w = W.conflict(trials=400, seed=21, grid=W.control_grid(4)[::3], reward=1.0, cost=0.1)
        d = cm.DeviceSweep(h, w, dumps=True)
        _wait(q, [q.submit(d)])
        g = d.results()
        correct = oracle.conflict_correct(w["weights"], w["params"][W.LCA_P["hid_gain"]],
                                          w["params"][W.LCA_P["hid_bias"]])
        assert_parity(w, g, oracle.run(w, dumps=True), correct)
    finally:
        q.close()


def test_queue_requests_joining_while_others_run():
    """Requests submitted one by one while earlier ones are still on the
    device, and eager launches of the program's own in between."""
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=16, idle_us=20000)
    try:
        ws = [W.conflict(trials=200 + 300 * i, seed=30 + i, grid=W.control_grid(4)[i::4],
                         precision=W.FP32_STEP) for i in range(10)]
        ds, tickets = [], []
        other = W.conflict(trials=500, seed=99, grid=W.control_grid(2))
        for i, w in enumerate(ws):
            d = cm.DeviceSweep(h, w)
            ds.append(d)
            tickets.append(q.submit(d))
            if i % 3 == 0:
                cm.run(other, handle=h)
        _wait(q, tickets)
        for i, (w, d) in enumerate(zip(ws, ds)):
            _same(d.results(), cm.run(w, handle=h), f"request {i}")
    finally:
        q.close()


def test_queue_kernel_ends_when_idle_and_comes_back():
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=4, idle_us=2000)
    try:
        for i in range(3):
            w = W.conflict(trials=300, seed=40 + i, grid=W.control_grid(2), precision=W.FP32_STEP)
            d = cm.DeviceSweep(h, w)
            _wait(q, [q.submit(d)])
            _same(d.results(), cm.run(w, handle=h), f"round {i}")
            time.sleep(0.05)  # the kernel has gone idle and ended; the next submit launches it again
    finally:
        q.close()


def test_queue_refuses_what_it_cannot_take():
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=1, idle_us=20000)
    try:
        w = W.conflict(trials=200, grid=W.control_grid(2), precision=W.FP32_STEP)
        d1, d2 = cm.DeviceSweep(h, w), cm.DeviceSweep(h, w)
        t1 = q.submit(d1)
        with pytest.raises(cm.CmError) as e:  # the one slot is held until its ticket is polled done
            q.submit(d2)
        assert e.value.status == cm.E_BUSY
        _wait(q, [t1])
        with pytest.raises(cm.CmError) as e:
            q.poll(t1)  # retired
        assert e.value.status == cm.E_INVALID
        with pytest.raises(cm.CmError) as e:
            q.submit(cm.DeviceSweep(h, W.ddm(trials=100)))
        assert e.value.status == cm.E_UNSUPPORTED
    finally:
        q.close()
    with pytest.raises(cm.CmError) as e:
        cm.DeviceQueue(h, W.DDM, W.FP64)
    assert e.value.status == cm.E_UNSUPPORTED


def test_queue_large_request_and_ring_reuse():
    """A request of 1250 chunks (the 64 x 10^4 conflict sweep), then more
    requests than the queue's ring holds (its entries are reused), four in
    flight at a time, each equal to cm_launch's."""
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=4, idle_us=20000)
    try:
        big = W.conflict(trials=10_000, seed=3, grid=W.control_grid(8), precision=W.FP32_STEP)
        d = cm.DeviceSweep(h, big)
        print("queue: 64 x 10^4 request", flush=True)
        _wait(q, [q.submit(d)])
        _same(d.results(), cm.run(big, handle=h), "large request")
        g = W.control_grid(2)
        ws = [W.conflict(trials=1 + i % 5, seed=500 + i, grid=g[i % 4:i % 4 + 1], precision=W.FP32_STEP)
              for i in range(1100)]
        print(f"queue: {len(ws)} small requests", flush=True)
        inflight, done = [], {}
        for i, w in enumerate(ws):
            dd = cm.DeviceSweep(h, w)
            while True:
                try:
                    inflight.append((i, dd, q.submit(dd)))
                    break
                except cm.CmError as e:
                    assert e.status == cm.E_BUSY
                    for j, dj, t in list(inflight):
                        if q.poll(t):
                            inflight.remove((j, dj, t))
                            done[j] = dj
        for j, dj, t in inflight:
            _wait(q, [t])
            done[j] = dj
        assert sorted(done) == list(range(len(ws)))
        for i in range(0, len(ws), 97):  # a sample against cm_launch
            _same(done[i].results(), cm.run(ws[i], handle=h), f"small request {i}")
    finally:
        q.close()


def test_queue_host_copies():
    """With pinned host buffers the kernel writes each request's hist, stats,
    score and best there before marking it done; pageable memory is refused."""
    import torch
    h = cm.Handle(0)
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=4, idle_us=20000)
    try:
        ws = [W.conflict(trials=300, seed=61, grid=W.control_grid(4), reward=1.0, cost=0.1, precision=W.FP32_STEP),
              W.conflict(trials=2000, seed=62, grid=W.control_grid(8)[::5], precision=W.FP32_STEP)]
        ds = [cm.DeviceSweep(h, w) for w in ws]
        hosts = [cm.host_buffers(d) for d in ds]
        for hh in hosts:
            for t in hh.values():
                t.fill_(7)
        tickets = [q.submit(d, host=hh) for d, hh in zip(ds, hosts)]
        _wait(q, tickets)
        for i, (w, hh) in enumerate(zip(ws, hosts)):
            ref = cm.run(w, handle=h)
            got = {k: (t.numpy().view(np.uint64) if k in ("hist", "stats") else t.numpy()) for k, t in hh.items()}
            for k in ("hist", "stats", "score", "best"):
                if ref.get(k) is not None:
                    assert np.array_equal(got[k], ref[k]), (i, k)
        d = cm.DeviceSweep(h, ws[1])
        pageable = {"hist": torch.empty(d.hist.shape, dtype=d.hist.dtype)}
        with pytest.raises(cm.CmError) as e:
            q.submit(d, host=pageable)
        assert e.value.status == cm.E_INVALID
    finally:
        q.close()


def test_queue_destroy_with_requests_in_flight():
    """Destroying a queue whose requests were never polled ends its kernel
    and returns; a new queue on the same handle then works as before."""
    h = cm.Handle(0)
    w = W.conflict(trials=3000, seed=71, grid=W.control_grid(4), precision=W.FP32_STEP)
    ds = [cm.DeviceSweep(h, W.with_(w, seed=71 + i)) for i in range(3)]
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=4, idle_us=20000)
    for d in ds:
        q.submit(d)
    print("queue: destroy with 3 requests in flight", flush=True)
    t0 = time.time()
    q.close()
    assert time.time() - t0 < 30.0
    q2 = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=4, idle_us=20000)
    try:
        d = cm.DeviceSweep(h, w)
        _wait(q2, [q2.submit(d)])
        _same(d.results(), cm.run(w, handle=h), "after a destroy")
    finally:
        q2.close()


def test_queue_large_grid_few_trials():
    """A 4,000-setting grid of 2 trials each (outcomes counted straight into
    global memory, many preparation pieces, the score and argmax over the
    whole grid in one workgroup) and a 2,000 x 50 scored grid, each equal to
    cm_launch's."""
    h = cm.Handle(0)
    g = W.control_grid(64)
    ws = [W.conflict(trials=2, seed=81, grid=g[:4000], reward=1.0, cost=0.1, precision=W.FP32_STEP),
          W.conflict(trials=50, seed=82, grid=g[:2000], reward=1.0, cost=0.1, precision=W.FP32_STEP)]
    q = cm.DeviceQueue(h, W.LCA, W.FP32_STEP, slots=4, idle_us=20000)
    try:
        ds = [cm.DeviceSweep(h, w, dumps=True) for w in ws]
        print("queue: large grids", flush=True)
        _wait(q, [q.submit(d) for d in ds])
        for i, (w, d) in enumerate(zip(ws, ds)):
            _same(d.results(), cm.run(w, dumps=True, handle=h), f"grid {i}")
    finally:
        q.close()
