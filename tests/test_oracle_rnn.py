"""Pins for the oracle's recurrent rate network."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W
import pins


def _drive_normals(w, setting, trial):
    """The per-run input drive: unit pair (2m, 2m+1) takes block m of the
    drive stream (pinned separately through the Philox and normal tests)."""
    nu = w["n_units"]
    u = np.zeros(nu)
    key = [w["seed"] & 0xFFFFFFFF, w["seed"] >> 32]
    for m in range(nu // 2):
        words = oracle.philox([m, trial, setting, 0x40000000], key)
        u[2 * m:2 * m + 2] = oracle.normals64(words)
    return u


def test_uncoupled_units_are_euler_ou_processes():
    """W = 0: each unit is x_n = (1-dt) x_{n-1} + dt g u + b xi; regressing
    x_n on the run's drive u gives the closed-form slope and residual
    variance."""
    nu, n, dt, noise, g = 8, 30, 0.05, 0.3, 1.7
    wts = np.zeros(nu * nu + 2 * nu)
    w = W.rnn(trials=6000, seed=3, n_units=nu, dt=dt, noise=noise, thresh=1e300,
              input_gain=g, max_steps=n, n_bins=10, weights=wts)
    out = oracle.run(w, dumps=True)
    x = out["run_state"][:, 2:]
    u = np.array([_drive_normals(w, 0, t) for t in range(6000)])
    slope, resid = pins.ou_moments(dt, noise * math.sqrt(dt), g, n)
    for i in range(nu):
        beta = (x[:, i] * u[:, i]).sum() / (u[:, i] ** 2).sum()
        r = x[:, i] - beta * u[:, i]
        assert abs(beta - slope) < 4.5 * math.sqrt(resid / (u[:, i] ** 2).sum())
        assert abs(r.var() / resid - 1) < 4.5 * math.sqrt(2 / r.size)


def test_noise_free_uncoupled_readout_closed_form():
    """W = 0, sigma = 0: x_n = g u (1 - (1-dt)^n) in closed form, and the
    readout integrates R (logistic(x_{n-1}) - 1/2) over the steps."""
    nu, n, dt, g = 16, 40, 0.05, 1.3
    rng = np.random.default_rng(4)
    R = rng.normal(0, 0.25, (2, nu))
    wts = np.concatenate([np.zeros(nu * nu), R.ravel()])
    w = W.rnn(trials=5, seed=8, n_units=nu, dt=dt, noise=0.0, thresh=1e300, input_gain=g,
              max_steps=n, n_bins=10, weights=wts)
    out = oracle.run(w, dumps=True)
    for t in range(5):
        u = _drive_normals(w, 0, t)
        y = np.zeros(2)
        for k in range(n):
            xk = g * u * (1 - (1 - dt) ** k)
            y = y + dt * (R @ (1 / (1 + np.exp(-xk)) - 0.5))
        xn = g * u * (1 - (1 - dt) ** n)
        np.testing.assert_allclose(out["run_state"][t, 2:], xn, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(out["run_state"][t, :2], y, rtol=1e-10, atol=1e-13)


def test_first_step_uses_rows_of_w():
    """From x = 0 every rate is 1/2, so after one noise-free step with no
    input x_1 = dt * W @ (1/2): the row sums of W (a transposed W would give
    column sums)."""
    nu = 32
    wts = W.rnn_weights(nu, 11)
    w = W.rnn(trials=1, n_units=nu, noise=0.0, input_gain=0.0, thresh=1e300, max_steps=1,
              n_bins=1, weights=wts)
    traj, _, _ = oracle.trajectory(w, 0, 0)
    Wm = wts[:nu * nu].reshape(nu, nu)
    np.testing.assert_allclose(traj[0, 2:], 0.05 * Wm.sum(1) * 0.5, rtol=1e-11, atol=1e-15)
    assert not np.allclose(traj[0, 2:], 0.05 * Wm.sum(0) * 0.5, rtol=1e-3)


def test_trajectory_and_sweep_agree():
    w = W.rnn(trials=6, seed=2, n_units=64, max_steps=200, weights=W.rnn_weights(64, 7))
    out = oracle.run(w, dumps=True)
    for t in range(6):
        traj, ch, fl = oracle.trajectory(w, 0, t)
        assert traj.shape[0] == out["run_step"][t]
        assert ch == out["run_choice"][t]
        np.testing.assert_array_equal(traj[-1], out["run_state"][t])


def test_decisions_and_invariants_at_reference_shape():
    """256 units with the reference weights: a substantial fraction of runs
    decides within 200 steps, both choices occur, undecided runs sit below
    threshold."""
    w = W.rnn(trials=256, seed=1)
    out = oracle.run(w, dumps=True, n_threads=8)
    st, hist = out["stats"][0], out["hist"][0]
    assert hist.sum() + st[oracle.ST["undec"]] == 256
    assert st[oracle.ST["dec0"]] > 10 and st[oracle.ST["dec1"]] > 10
    y = out["run_state"][:, :2]
    dec = out["run_choice"] >= 0
    assert np.all(y[dec].max(1) >= 1.0) and np.all(y[~dec].max(1) < 1.0)
    assert st[oracle.ST["correct"]] == 0  # the rate network defines no correct response


@pytest.mark.parametrize("prec", [W.FP32_STEP, W.BF16_PROJ])
def test_reduced_precision_close_to_fp64(prec):
    w = W.rnn(trials=512, seed=5, n_units=64, weights=W.rnn_weights(64, 7) * 2.0)
    a = oracle.run(w, dumps=True, n_threads=8)
    b = oracle.run(W.with_(w, precision=prec), dumps=True, n_threads=8)
    agree = (a["run_choice"] == b["run_choice"]).mean()
    assert agree > 0.95
    pa = a["hist"][0] / 512
    pb = b["hist"][0] / 512
    assert np.abs(pa.sum(1) - pb.sum(1)).max() < 0.03


def test_coupled_network_settles_at_its_fixed_point():
    """Noise-free, no input, two groups of four units coupled within and
    across groups with different strengths each way: from x = 0 every unit
    of a group follows the same path, and the network settles where
    x_A = a s(x_A) + c_AB s(x_B) and x_B = c_BA s(x_A) + b s(x_B) (s the
    logistic; the fixed point of the continuous dynamics, found here by root
    finding).  A transposed W would exchange c_AB and c_BA."""
    from scipy.optimize import fsolve
    a, b, c_ab, c_ba = 1.0, -0.5, 0.8, -0.6
    nu = 8
    Wm = np.zeros((nu, nu))
    A, B = range(0, 4), range(4, 8)
    for i in A:
        for j in A:
            if j != i:
                Wm[i, j] = a / 3
        for j in B:
            Wm[i, j] = c_ab / 4
    for i in B:
        for j in A:
            Wm[i, j] = c_ba / 4
        for j in B:
            if j != i:
                Wm[i, j] = b / 3
    wts = np.concatenate([Wm.ravel(), np.zeros(2 * nu)])
    w = W.rnn(trials=2, seed=5, n_units=nu, dt=0.05, noise=0.0, thresh=1e300, input_gain=0.0,
              max_steps=1500, n_bins=10, weights=wts)
    out = oracle.run(w, dumps=True)

    def s(x):
        return 1.0 / (1.0 + np.exp(-x))

    xa, xb = fsolve(lambda v: [v[0] - a * s(v[0]) - c_ab * s(v[1]),
                               v[1] - c_ba * s(v[0]) - b * s(v[1])], [0.5, -0.5], xtol=1e-14)
    swapped = fsolve(lambda v: [v[0] - a * s(v[0]) - c_ba * s(v[1]),
                                v[1] - c_ab * s(v[0]) - b * s(v[1])], [0.5, -0.5], xtol=1e-14)
    assert abs(swapped[0] - xa) > 0.1
    for t in range(2):
        x = out["run_state"][t, 2:]
        np.testing.assert_allclose(x[:4], xa, rtol=0, atol=1e-9)
        np.testing.assert_allclose(x[4:], xb, rtol=0, atol=1e-9)
    assert np.all(out["stats"][:, 2] == 2)  # undecided at the cap
