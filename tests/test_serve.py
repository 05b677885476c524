"""Serving scheduler on the CPU with a simulated device: admission by memory
budget, stream slots, batching, completion accounting."""
import numpy as np
import pytest

from paper_2110_15425_amd import serve, workloads as W


class FakeBackend:
    """Completes a launched group after `delay` polls; records what ran."""

    def __init__(self, delay=3):
        self.t = 0.0
        self.delay = delay
        self.launches = []
        self.peak_inflight = 0
        self.live = 0

    def clock(self):
        self.t += 1e-4
        return self.t

    def launch(self, si, ws):
        self.launches.append((si, len(ws)))
        self.live += 1
        self.peak_inflight = max(self.peak_inflight, self.live)
        return {"left": self.delay, "n": len(ws)}

    def poll(self, token):
        token["left"] -= 1
        if token["left"] > 0:
            return None
        self.live -= 1
        return [{"stats": np.zeros((1, 9), np.uint64)} for _ in range(token["n"])]


def _reqs(n, trials=1000):
    return [serve.Request(i, W.ddm(trials=trials + i, seed=i), 0.0) for i in range(n)]


def test_all_requests_finish_and_budget_holds():
    be = FakeBackend()
    reqs = _reqs(40)
    budget = 3 * max(r.nbytes for r in reqs)
    sch = serve.Scheduler(be, budget, n_streams=2, max_group=4)
    peak = 0
    for r in reqs:
        sch.submit(r)
    while not sch.idle():
        sch.tick()
        peak = max(peak, sch.used)
        assert sch.used <= budget
    assert peak > 0 and sch.used == 0
    assert sorted(r.rid for r in sch.finished) == list(range(40))
    assert all(r.done >= r.admitted >= r.arrival for r in sch.finished)
    assert be.peak_inflight <= 2
    assert max(n for _, n in be.launches) <= 4


def test_oversized_request_rejected():
    be = FakeBackend()
    r = _reqs(1)[0]
    sch = serve.Scheduler(be, r.nbytes - 1)
    with pytest.raises(ValueError):
        sch.submit(r)


def test_small_requests_pass_a_large_waiting_one():
    be = FakeBackend(delay=50)
    big = serve.Request(0, W.grid_search(), 0.0)
    small = [serve.Request(i + 1, W.ddm(trials=10, seed=i), 0.0) for i in range(3)]
    first = serve.Request(9, W.grid_search(seed=2), 0.0)
    budget = first.nbytes + sum(s.nbytes for s in small) + 1024
    sch = serve.Scheduler(be, budget, n_streams=4)
    sch.submit(first)
    sch.tick()  # first is in flight, holding most of the budget
    sch.submit(big)
    for s in small:
        sch.submit(s)
    sch.tick()
    admitted = {r.rid for r in small if r.admitted is not None}
    assert admitted == {1, 2, 3} and big.admitted is None
    sch.drain(sleep=0)
    assert big.done is not None


def test_served_mix_recipe():
    mix = serve.served_mix(400, rate_hz=50.0, seed=11)
    t = np.array([a for a, _ in mix])
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 50.0) < 10.0  # Poisson rate
    kinds = [w["kind"] for _, w in mix]
    assert set(kinds) == {0, 1, 2}
    for _, w in mix:
        runs = w["n_settings"] * w["trials"]
        assert 1 <= w["n_settings"] <= 4096
        assert runs >= 1 and w["trials"] >= 1
        assert w["seed"] >= 1000


def test_latency_by_config_groups_requests_by_model_configuration():
    """Each served request belongs to exactly one of the four configurations,
    and the per-configuration summaries cover every finished request."""
    mix = serve.served_mix(200, rate_hz=50.0, seed=11)
    names = [serve.CONFIG_NAMES[serve.config_of(w)] for _, w in mix]
    assert set(names) == set(serve.CONFIG_NAMES.values())

    class Done:
        def __init__(self, w, lat):
            self.w, self.arrival, self.done = w, 0.0, lat

    finished = [Done(w, 0.001 * (1 + i % 7)) for i, (_, w) in enumerate(mix)]
    by = serve.latency_by_config(finished)
    assert sum(v["requests"] for v in by.values()) == len(finished)
    for name, v in by.items():
        assert v["requests"] == names.count(name)
        assert 1.0 <= v["p50_ms"] <= v["p99_ms"] <= v["max_ms"] <= 7.0
