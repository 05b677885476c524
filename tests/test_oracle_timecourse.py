"""Pins for the oracle's ensemble time course (count and fixed-point sums of
the state, its squares and the conflict energy at sample steps)."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W
import pins

S32 = 2.0 ** 32


def test_quantisation_rounds_half_to_even_and_clamps():
    assert oracle.tc_quant(1.0) == 1 << 32
    assert oracle.tc_quant(-0.5) == -(1 << 31)
    assert oracle.tc_quant(2.0 ** -33) == 0          # 0.5 quantum -> even 0
    assert oracle.tc_quant(3 * 2.0 ** -33) == 2      # 1.5 quanta -> even 2
    assert oracle.tc_quant(-3 * 2.0 ** -33) == -2
    assert oracle.tc_quant(1e30) == 1 << 62
    assert oracle.tc_quant(-1e30) == -(1 << 62)


def test_noise_free_ddm_follows_the_straight_line_and_drops_out_at_the_crossing():
    """sigma = 0: every run is x_n = n a until the first n with n a >= theta
    (n* = 334 for a = 0.003, theta = 1); samples after n* see no run."""
    T, every = 37, 10
    w = W.ddm(trials=T, noise=0.0, drift=0.3, dt=0.01, max_steps=400)
    tc = oracle.timecourse(w, every)
    assert tc.shape == (1, 40, 6)
    for k in range(1, 41):
        n = k * every
        row = tc[0, k - 1]
        if n <= 334:
            assert row[0] == T
            assert abs(row[1] / S32 / T - n * 0.003) < 1e-9, n
            assert abs(row[3] / S32 / T - (n * 0.003) ** 2) < 1e-9, n
        else:
            assert row[0] == 0 and row[1] == 0 and row[3] == 0
        assert row[2] == row[4] == row[5] == 0  # one unit


def test_gaussian_walk_moments():
    """Threshold out of reach: x_n = n a + b (z_1 + ... + z_n) is exactly
    N(n a, n b^2)."""
    T, every, N = 20000, 20, 200
    a, b = 0.3 * 0.01, 1.0 * 0.1
    w = W.ddm(trials=T, thresh=1e6, max_steps=N, n_bins=10, seed=3)
    tc = oracle.timecourse(w, every)
    cnt, mom = oracle.tc_moments(tc)
    for k in range(N // every):
        n = (k + 1) * every
        assert cnt[0, k] == T
        mean, var = n * a, n * b * b
        m1, m2 = mom[0, k, 0], mom[0, k, 2]
        assert abs(m1 - mean) < 5 * math.sqrt(var / T), (n, m1, mean)
        v = m2 - m1 * m1
        assert abs(v - var) < 5 * var * math.sqrt(2.0 / T), (n, v, var)


def _mixture_moments(drive, leak, comp, dt, b, n):
    """Mean vector and second moments E[x0^2], E[x1^2], E[x0 x1] of the
    equal-weight mixture over the nine stimuli, and their sampling variances
    per run (Gaussian fourth moments, Isserlis)."""
    mus, covs = [], []
    for stim in range(9):
        m, C = pins.lca_linear_moments(drive[stim], leak, comp, dt, b, n)
        mus.append(np.asarray(m))
        covs.append(np.asarray(C))
    first = np.mean(mus, 0)
    sec = np.mean([C + np.outer(m, m) for m, C in zip(mus, covs)], 0)
    # E[Y^2] for Y = x0, x0^2, x1^2, x0 x1, averaged over stimuli
    def fourth(m, C):
        m0, m1 = m
        s00, s11, s01 = C[0, 0], C[1, 1], C[0, 1]
        e_x0sq_sq = m0 ** 4 + 6 * m0 ** 2 * s00 + 3 * s00 ** 2
        e_x1sq_sq = m1 ** 4 + 6 * m1 ** 2 * s11 + 3 * s11 ** 2
        e_x0x1_sq = (m0 ** 2 * m1 ** 2 + m0 ** 2 * s11 + m1 ** 2 * s00 + 4 * m0 * m1 * s01
                     + s00 * s11 + 2 * s01 ** 2)
        return np.array([s00 + m0 ** 2, s11 + m1 ** 2, e_x0sq_sq, e_x1sq_sq, e_x0x1_sq])
    f = np.mean([fourth(m, C) for m, C in zip(mus, covs)], 0)
    ex = np.array([first[0], first[1], sec[0, 0], sec[1, 1], sec[0, 1]])
    var = f - ex ** 2
    return ex, var


@pytest.mark.parametrize("leak,comp", [(0.5, 1.0), (0.3, 0.3)])
def test_linear_lca_mixture_moments(leak, comp):
    """Threshold out of reach: each stimulus' state is Gaussian with the
    linear recursion's moments; the time course averages the nine."""
    T, every, N, dt, noise = 9 * 2000, 5, 30, 0.1, 0.4
    w = W.conflict(trials=T, seed=22, leak=leak, comp=comp, noise=noise, thresh=1e300, dt=dt,
                   max_steps=N, n_bins=3, grid=np.array([[0.8, 1.3]]))
    tc = oracle.timecourse(w, every)
    cnt, mom = oracle.tc_moments(tc)
    drive = oracle.conflict_drive(w["weights"], 1.0, -4.0, 0.0, 0.8, 1.3)
    b = noise * math.sqrt(dt)
    for k in range(N // every):
        n = (k + 1) * every
        assert cnt[0, k] == T
        ex, var = _mixture_moments(drive, leak, comp, dt, b, n)
        got = np.array([mom[0, k, 0], mom[0, k, 1], mom[0, k, 2], mom[0, k, 3],
                        mom[0, k, 4] / comp])
        se = np.sqrt(var / T)
        assert np.all(np.abs(got - ex) < 5 * se), (n, got, ex, se)


def test_survival_matches_first_passage_density():
    """Count at step n = runs not decided before n; its expectation is T
    times the survival of the exact discrete-walk density."""
    T, every = 10000, 30
    w = W.ddm(trials=T)
    tc = oracle.timecourse(w, every)
    lo, up = oracle.ddm_density(0.003, 0.1, 1.0, cells=1000, max_steps=3000)
    F = np.concatenate([[0.0], np.cumsum(lo + up)])  # F[m] = P(decided by step m)
    for k in range(100):
        n = (k + 1) * every
        p = 1.0 - F[n - 1]
        sd = math.sqrt(max(p * (1 - p), 1e-12) / T)
        assert abs(tc[0, k, 0] / T - p) < 5 * sd + 1e-12, (n, tc[0, k, 0] / T, p)


@pytest.mark.parametrize("kind", ["ddm", "lca"])
def test_counts_agree_with_per_run_decision_steps(kind):
    """An independent route to the counts: the per-run decision steps of
    cmo_run, counted at each sample step."""
    if kind == "ddm":
        w = W.ddm(trials=3000, drifts=[0.1, 0.3, 0.8], max_steps=600)
        every = 7
    else:
        w = W.conflict(trials=450, grid=W.control_grid(4)[:5], max_steps=200)
        every = 3
    tc = oracle.timecourse(w, every)
    out = oracle.run(w, dumps=True)
    steps = out["run_step"].reshape(int(w["n_settings"]), -1)
    K = int(w["max_steps"]) // every
    for s in range(int(w["n_settings"])):
        for k in range(K):
            assert tc[s, k, 0] == int((steps[s] >= (k + 1) * every).sum())


def test_last_sample_and_cap():
    """every that does not divide max_steps: K = floor(N / every), and
    undecided runs contribute at every sample up to the cap."""
    w = W.ddm(trials=50, thresh=1e6, max_steps=23, n_bins=5)
    tc = oracle.timecourse(w, 5)
    assert tc.shape == (1, 4, 6)
    assert np.all(tc[0, :, 0] == 50)
    with pytest.raises(ValueError):
        oracle.timecourse(w, 24)
    with pytest.raises(ValueError):
        oracle.timecourse(W.rnn(trials=4, n_units=4, max_steps=5, n_bins=5), 1)
