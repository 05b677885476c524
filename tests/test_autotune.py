"""Host logic of the launch-shape autotuner: size classes, cache keys and
candidate lists (no GPU)."""
from paper_2110_15425_amd import autotune, workloads as W


def test_size_class_buckets_by_powers_of_two():
    w = W.conflict(trials=10_000)
    assert autotune.size_class(w) == "S6-T13-N9"  # 64 settings, 10^4 trials, cap 1000
    assert autotune.size_class(W.with_(w, trials=16_383)) == "S6-T13-N9"
    assert autotune.size_class(W.with_(w, trials=16_384)) == "S6-T14-N9"
    assert autotune.size_class(W.ddm(trials=1)).startswith("S0-T0-")


def test_cache_key_separates_kind_precision_and_device():
    w = W.conflict(trials=10_000)
    k = autotune.cache_key(w, "gpu")
    assert k != autotune.cache_key(W.with_(w, precision=W.FP32_STEP), "gpu")
    assert k != autotune.cache_key(w, "other")
    assert k != autotune.cache_key(W.ddm(trials=10_000), "gpu")
    assert k == autotune.cache_key(W.with_(w, seed=99), "gpu")  # seeds share shapes


def test_default_candidates():
    lca = autotune.default_candidates(W.conflict())
    assert len(lca) == len(autotune.RUNS_PER_LANE) * len(autotune.STEPS_PER_SYNC)
    assert all(c[2] == 1 for c in lca)
    ddm = autotune.default_candidates(W.ddm())
    wave = [c for c in ddm if c[2] == 64]  # one wavefront per run
    assert [c[0] for c in wave] == list(autotune.RUNS_PER_WAVE)
    assert len(ddm) == len(lca) + len(wave)
