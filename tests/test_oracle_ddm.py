"""Pins for the oracle's drift-diffusion runs (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W
import pins


@pytest.fixture(scope="module")
def density():
    # the first configuration: drift 0.3, sd 1, threshold 1, dt 0.01
    return pins.ddm_walk_density(0.3 * 0.01, 1.0 * math.sqrt(0.01), 1.0, max_steps=3000)


def test_density_helper_against_closed_form(density):
    """The propagation itself agrees with the boundary-shifted continuous
    first-passage formulas (Broadie-Glasserman-Kou), which are accurate to
    O(dt) -- this guards the pin, not the oracle."""
    up, lo = density
    n = np.arange(1, up.size + 1)
    p_err, mean_dt = pins.ddm_bgk(0.3, 1.0, 1.0, 0.01)
    assert lo.sum() == pytest.approx(p_err, abs=2e-4)
    assert ((up + lo) * n).sum() * 0.01 == pytest.approx(mean_dt, abs=5e-3)
    assert up.sum() + lo.sum() == pytest.approx(1.0, abs=1e-9)


@pytest.mark.parametrize("seed", [1, 2])
def test_histogram_matches_first_passage_density(density, seed):
    up, lo = density
    w = W.ddm(trials=100_000, seed=seed)
    out = oracle.run(w)
    hist = out["hist"][0]
    st = out["stats"][0]
    assert st[oracle.ST["undec"]] == 0
    expected = np.concatenate([pins.binned(lo, 100, 3000), pins.binned(up, 100, 3000)])
    observed = np.concatenate([hist[0], hist[1]])
    assert pins.chisq_pvalue(observed, expected) > 1e-4
    T = w["trials"]
    p_up = st[oracle.ST["dec1"]] / T
    se = math.sqrt(up.sum() * (1 - up.sum()) / T)
    assert abs(p_up - up.sum()) < 4 * se
    n = np.arange(1, up.size + 1)
    mean_n = ((up + lo) * n).sum()
    sd_n = math.sqrt(((up + lo) * n * n).sum() - mean_n ** 2)
    got = (st[oracle.ST["sumn0"]] + st[oracle.ST["sumn1"]]) / T
    assert abs(got - mean_n) < 4 * sd_n / math.sqrt(T)


def test_fp32_steps_follow_the_same_density(density):
    up, lo = density
    w = W.ddm(trials=100_000, seed=3, precision=W.FP32_STEP)
    hist = oracle.run(w)["hist"][0]
    expected = np.concatenate([pins.binned(lo, 100, 3000), pins.binned(up, 100, 3000)])
    assert pins.chisq_pvalue(np.concatenate([hist[0], hist[1]]), expected) > 1e-4


def test_other_setting_density():
    """A second parameter point (negative drift, biased start, coarse dt)."""
    a, b, th = -0.2 * 0.05, 0.7 * math.sqrt(0.05), 0.6
    up, lo = pins.ddm_walk_density(a, b, th, start=0.15, max_steps=400, cells=600)
    w = W.ddm(trials=50_000, seed=4, drift=-0.2, noise=0.7, thresh=0.6, start=0.15, dt=0.05,
              max_steps=400, n_bins=40)
    out = oracle.run(w)
    hist, st = out["hist"][0], out["stats"][0]
    exp = np.concatenate([pins.binned(lo, 40, 400), pins.binned(up, 40, 400)])
    # undecided runs carry the missing mass
    p_undec = max(0.0, 1 - up.sum() - lo.sum())
    obs = np.concatenate([hist[0], hist[1], [st[oracle.ST["undec"]]]])
    assert pins.chisq_pvalue(obs, np.concatenate([exp, [p_undec]])) > 1e-4


@pytest.mark.parametrize("drift,choice", [(0.3, 1), (-0.3, 0)])
def test_noise_free_crossing_step(drift, choice):
    """sigma = 0: x_n is the running FP64 sum of a = drift*dt, so the decision
    step is the first n whose sum passes the bound (brute force)."""
    a = drift * 0.01
    x, n = 0.0, 0
    while -1.0 < x < 1.0:
        x = x + a
        n += 1
    w = W.ddm(trials=50, noise=0.0, drift=drift)
    out = oracle.run(w, dumps=True)
    assert n == 334
    assert set(out["run_step"]) == {n}
    assert set(out["run_choice"]) == {choice}
    assert np.all(out["run_state"][:, 0] == x)


def test_cap_and_undecided():
    w = W.ddm(trials=2000, noise=0.0, drift=0.0, max_steps=50, n_bins=10)
    out = oracle.run(w, dumps=True)
    st = out["stats"][0]
    assert st[oracle.ST["undec"]] == 2000 and out["hist"].sum() == 0
    assert set(out["run_choice"]) == {-1} and set(out["run_step"]) == {50}
    # the default "correct" response is the upper boundary; undecided are not correct
    assert st[oracle.ST["correct"]] == 0


def test_drift_grid_settings_are_independent_and_invariants_hold():
    drifts = np.linspace(0.0, 0.6, 7)
    w = W.ddm(trials=3000, seed=11, drifts=drifts)
    out = oracle.run(w, dumps=True)
    hist, st = out["hist"], out["stats"]
    T = w["trials"]
    assert np.all(hist.sum(axis=(1, 2)) + st[:, oracle.ST["undec"]] == T)
    assert np.all(st[:, oracle.ST["correct"]] == st[:, oracle.ST["dec1"]])
    # larger drift -> more upper crossings
    p1 = st[:, oracle.ST["dec1"]] / T
    assert np.all(np.diff(p1) > 0)
    # sum of decision steps within the bounds implied by the bins (30 steps each)
    for s in range(7):
        for c in (0, 1):
            lo = (hist[s, c] * (np.arange(100) * 30 + 1)).sum()
            hi = (hist[s, c] * (np.arange(100) * 30 + 30)).sum()
            assert lo <= st[s, oracle.ST["sumn0"] + c] <= hi
    # per-run dumps reduce to the same statistics
    ch = out["run_choice"].reshape(7, T)
    stp = out["run_step"].reshape(7, T).astype(np.uint64)
    for s in range(7):
        assert st[s, oracle.ST["sumsq1"]] == (stp[s][ch[s] == 1] ** 2).sum()
    # the thread count does not change any integer output
    w2 = W.ddm(trials=3000, seed=11, drifts=drifts)
    again = oracle.run(w2, n_threads=3)
    assert np.array_equal(again["hist"], hist) and np.array_equal(again["stats"], st)


def test_flag_marks_near_threshold_runs():
    # with a huge epsilon every executed step is "near", so every run is flagged
    w = W.ddm(trials=500, flag_eps=10.0)
    out = oracle.run(w, dumps=True)
    assert out["stats"][0, oracle.ST["flagged"]] == 500 and out["run_flag"].all()
    # with the default epsilon a flag is rare (expected ~1e-8 per run)
    out = oracle.run(W.ddm(trials=20_000))
    assert out["stats"][0, oracle.ST["flagged"]] == 0


# --- the oracle's density propagation (the exact first-passage distribution) ---

def test_density_oracle_against_independent_propagation_and_closed_form(density):
    lo, up = oracle.ddm_density(0.3 * 0.01, 0.1, 1.0, cells=1000, max_steps=3000)
    u2, l2 = density  # scipy/numpy implementation in tests/pins.py
    np.testing.assert_allclose(up, u2, rtol=0, atol=1e-14)
    np.testing.assert_allclose(lo, l2, rtol=0, atol=1e-14)
    assert up.sum() + lo.sum() == pytest.approx(1.0, abs=1e-12)
    p_err, mean_dt = pins.ddm_bgk(0.3, 1.0, 1.0, 0.01)
    n = np.arange(1, 3001)
    assert lo.sum() == pytest.approx(p_err, abs=2e-4)
    assert ((up + lo) * n).sum() * 0.01 == pytest.approx(mean_dt, abs=5e-3)


def test_density_oracle_matches_monte_carlo_oracle():
    """Biased start and negative drift: the density's binned probabilities
    explain the Monte-Carlo oracle's 2*10^5-trial histogram."""
    a, b, th, x0 = -0.1 * 0.02, 0.8 * math.sqrt(0.02), 0.7, 0.2
    lo, up = oracle.ddm_density(a, b, th, start=x0, cells=700, max_steps=600)
    w = W.ddm(trials=200_000, seed=8, drift=-0.1, noise=0.8, thresh=0.7, start=0.2, dt=0.02,
              max_steps=600, n_bins=60)
    out = oracle.run(w, n_threads=8)
    exp = np.concatenate([pins.binned(lo, 60, 600), pins.binned(up, 60, 600),
                          [max(0.0, 1 - lo.sum() - up.sum())]])
    obs = np.concatenate([out["hist"][0, 0], out["hist"][0, 1], [out["stats"][0, 2]]])
    assert pins.chisq_pvalue(obs, exp) > 1e-4


def test_density_oracle_early_stop_and_rejects():
    lo, up = oracle.ddm_density(0.05, 0.2, 0.5, cells=200, max_steps=2000, tol=1e-12)
    last = np.flatnonzero(up + lo)[-1]
    assert last < 1999 and np.all(up[last + 1:] == 0) and np.all(lo[last + 1:] == 0)
    assert up.sum() + lo.sum() == pytest.approx(1.0, abs=1e-11)
    with pytest.raises(ValueError):
        oracle.ddm_density(0.0, 0.0, 1.0)  # no noise: no density
