"""Pins for the oracle's closed-loop control of the conflict network: the
control search nested in every step reduces to the (pinned) open-loop LCA when
only one allocation exists or control is prohibitively expensive, and with no
noise it follows the argmin of the look-ahead's closed-form expectation."""
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W


def _same_runs(a, b):
    assert np.array_equal(a["run_choice"], b["run_choice"])
    assert np.array_equal(a["run_step"], b["run_step"])
    assert np.array_equal(a["run_state"], b["run_state"])
    assert np.array_equal(a["hist"], b["hist"])
    assert np.array_equal(a["stats"][:, :8], b["stats"][:, :8])


@pytest.mark.parametrize("prec", [W.FP64, W.FP32_STEP])
def test_single_allocation_is_the_open_loop_lca(prec):
    """L = 1: the only allocation is (A_max, A_max), and the executed step uses
    the run's own stream, so every run equals the open-loop LCA run."""
    loop = W.control_loop(trials=450, levels=1, amax=1.7, samples=3, costs=[0.0, 0.5],
                          precision=prec)
    lca = W.conflict(trials=450, grid=np.array([[1.7, 1.7], [1.7, 1.7]]), precision=prec)
    _same_runs(oracle.run(loop, dumps=True), oracle.run(lca, dumps=True))


def test_prohibitive_cost_keeps_control_off():
    """With a cost weight far above any look-ahead gain the cheapest
    allocation (0, 0) wins every step: the open-loop LCA at zero control."""
    loop = W.control_loop(trials=270, levels=6, samples=2, costs=[1e6])
    lca = W.conflict(trials=270, grid=np.array([[0.0, 0.0]]))
    _same_runs(oracle.run(loop, dumps=True), oracle.run(lca, dumps=True))


def _noise_free_prediction(w, stim):
    """Deterministic controlled recursion with the look-ahead's expectation in
    closed form: gain_j = dt ((I_c - I_w)(j) + (comp - leak)(x_c - x_w))."""
    p = w["params"]
    P = W.LOOP_P
    dt, leak, comp, th = p[P["dt"]], p[P["leak"]], p[P["comp"]], p[P["thresh"]]
    L, amax, kappa = int(p[P["levels"]]), p[P["amax"]], float(w["grid"][0, 0])
    lv = amax * np.arange(L) / (L - 1)
    cA, cB = np.repeat(lv, L), np.tile(lv, L)
    drives = np.array([oracle.conflict_drive(w["weights"], p[P["hid_gain"]], p[P["hid_bias"]],
                                             p[P["offset"]], a, b)[stim] for a, b in zip(cA, cB)])
    c = oracle.conflict_correct(w["weights"], p[P["hid_gain"]], p[P["hid_bias"]])[stim]
    o = 1 - c
    x = np.zeros(2)
    for n in range(1, int(w["max_steps"]) + 1):
        gain = dt * ((drives[:, c] - drives[:, o]) + (comp - leak) * (x[c] - x[o]))
        V = kappa * (cA * cA + cB * cB) - gain
        order = np.argsort(V)
        if V[order[1]] - V[order[0]] < 1e-9:
            return None  # too close to call in floating point
        I = drives[order[0]]
        x = np.array([x[0] + (I[0] - leak * x[0] - comp * x[1]) * dt,
                      x[1] + (I[1] - leak * x[1] - comp * x[0]) * dt])
        if x.max() >= th:
            return n, int(x[1] > x[0])
    return int(w["max_steps"]), -1


@pytest.mark.parametrize("kappa", [0.0, 0.01, 0.05])
def test_noise_free_control_follows_the_expected_gain(kappa):
    w = W.control_loop(trials=9, levels=5, samples=2, noise=0.0, costs=[kappa], max_steps=400)
    out = oracle.run(w, dumps=True)
    checked = 0
    for stim in range(9):
        pred = _noise_free_prediction(w, stim)
        if pred is None:
            continue
        checked += 1
        assert (int(out["run_step"][stim]), int(out["run_choice"][stim])) == pred, stim
    assert checked >= 6


def test_invariants():
    w = W.control_loop(trials=91, levels=4, samples=3, costs=[0.0, 0.01, 0.1], max_steps=60,
                       n_bins=7)
    out = oracle.run(w, dumps=True)
    st = out["stats"].astype(np.int64)
    T = int(w["trials"])
    assert np.all(out["hist"].sum(axis=(1, 2)) + st[:, 2] == T)
    assert np.all(st[:, 3] <= st[:, 0] + st[:, 1])
    assert np.all(st[:, 0] + st[:, 1] + st[:, 2] == T)
    ch = out["run_choice"].reshape(3, T)
    assert np.array_equal((ch == 0).sum(1), st[:, 0])


def test_rejects_bad_search_shapes():
    for bad in (dict(levels=0), dict(levels=2.5), dict(samples=0), dict(levels=4096, samples=100)):
        with pytest.raises(ValueError):
            oracle.run(W.control_loop(trials=2, max_steps=3, n_bins=1, **bad))
