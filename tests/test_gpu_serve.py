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


def test_budget_smaller_than_mix_still_completes():
    h = cm.Handle(0)
    mix = serve.served_mix(16, rate_hz=1e6, seed=6, max_runs=10_000)
    biggest = max(serve.request_bytes(w) for _, w in mix)
    done = serve.run_mix(h, mix, budget_bytes=biggest + 1, n_streams=2)
    assert len(done) == 16
