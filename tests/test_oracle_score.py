"""Pins for the grid score and the random tie-break among best settings."""
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W


def _tie_pick(seed, candidates):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    pr = [(int(oracle.philox([0, s, 0xFFFFFFFF, 0xFFFFFFFF], key)[0]), s) for s in candidates]
    return min(pr)[1]


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_forced_ties_pick_by_priority(seed):
    """Noise-free runs make duplicated settings score identically; the pick
    is the tie with the smallest stream priority, whatever the order."""
    base = np.array([[0.5, 1.0], [0.5, 1.0], [1.0, 0.5], [0.5, 1.0], [1.0, 0.5], [2.0, 2.0]])
    w = W.conflict(trials=27, seed=seed, noise=0.0, grid=base, reward=1.0, cost=0.0)
    out = oracle.run(w)
    sc = out["score"]
    best = sc.max()
    ties = [s for s in range(len(base)) if sc[s] == best]
    assert len(ties) >= 2
    assert out["best"][1] == len(ties)
    assert out["best"][0] == _tie_pick(seed, ties)


def test_tie_pick_is_uniform():
    """Over many seeds each of k tied settings is picked about 1/k of the time."""
    k, n = 4, 4000
    counts = np.zeros(k)
    for seed in range(n):
        counts[_tie_pick(seed, range(k))] += 1
    assert np.all(np.abs(counts / n - 1 / k) < 4 * np.sqrt((1 / k) * (1 - 1 / k) / n))


def test_grid_scores_against_integer_key():
    """On the 64x64 grid with 100 trials, reward 1 and cost 0.1 the score is
    (3969 correct - 250 (i^2 + j^2)) / 396900 exactly; FP64 ties must be
    real ties and distinct keys must order the same way."""
    w = W.grid_search(trials=100, seed=1, max_steps=1000)
    out = oracle.run(w, n_threads=8)
    corr = out["stats"][:, oracle.ST["correct"]].astype(np.int64)
    i, j = np.divmod(np.arange(4096), 64)
    key = 3969 * corr - 250 * (i * i + j * j)
    sc = out["score"]
    np.testing.assert_allclose(sc, key / 396900.0, rtol=0, atol=4e-15)  # a few ulp at |score| <= 5
    order = np.argsort(key, kind="stable")
    ks, ss = key[order], sc[order]
    distinct = np.diff(ks) > 0
    assert np.all(np.diff(ss)[distinct] > 0)
    best_key = key.max()
    fp_ties = np.flatnonzero(sc == sc.max())
    assert np.all(key[fp_ties] == best_key)
    assert out["best"][0] in fp_ties and out["best"][1] == fp_ties.size
    assert out["best"][0] == _tie_pick(1, fp_ties)


def test_score_formula_small_grid():
    grid = np.array([[0.0, 0.0], [1.0, 2.0], [3.0, 0.5]])
    w = W.conflict(trials=90, seed=3, grid=grid, reward=2.0, cost=0.3)
    out = oracle.run(w)
    corr = out["stats"][:, oracle.ST["correct"]]
    for s in range(3):
        pen = grid[s, 0] * grid[s, 0] + grid[s, 1] * grid[s, 1]
        assert out["score"][s] == 2.0 * (corr[s] / 90.0) - 0.3 * pen


def test_no_score_without_reward_or_cost():
    out = oracle.run(W.conflict(trials=9, grid=np.array([[1.0, 1.0]])))
    assert out["score"] is None and out["best"] is None
