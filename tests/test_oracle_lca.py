"""Pins for the oracle's conflict network and leaky competing accumulator."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W
import pins


def _torch_drive(weights, gain, bias, offset, cA, cB):
    """The conflict network's feed-forward pass as a PyTorch two-layer net:
    one-hot inputs -> logistic hidden layers (gain scaled by the control
    signal) -> linear projections onto the two accumulators."""
    import torch
    wt = torch.tensor(weights, dtype=torch.float64)
    WA, WB = wt[:12].view(4, 3), wt[12:24].view(4, 3)
    OA, OB = wt[24:32].view(2, 4), wt[32:40].view(2, 4)
    eye = torch.eye(3, dtype=torch.float64)
    out = torch.zeros(9, 2, dtype=torch.float64)
    for stim in range(9):
        a, b = divmod(stim, 3)
        hA = torch.sigmoid(cA * gain * (torch.nn.functional.linear(eye[a], WA) + bias))
        hB = torch.sigmoid(cB * gain * (torch.nn.functional.linear(eye[b], WB) + bias))
        out[stim] = torch.nn.functional.linear(hA, OA) + torch.nn.functional.linear(hB, OB) + offset
    return out.numpy()


@pytest.mark.parametrize("wseed", [7, 8, 9])
@pytest.mark.parametrize("cA,cB", [(0.0, 0.0), (1.0, 1.0), (5 * 17 / 63, 1.0), (5.0, 2.5)])
def test_drive_matches_torch_network(wseed, cA, cB):
    wt = W.conflict_weights(wseed)
    got = oracle.conflict_drive(wt, 1.0, -4.0, 0.25, cA, cB)
    want = _torch_drive(wt, 1.0, -4.0, 0.25, cA, cB)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)


def test_drive_special_case_zero_control():
    """c = 0: every hidden unit sits at logistic(0) = 1/2, so the drive is
    half the row sums of the projections, for every stimulus."""
    wt = W.conflict_weights(7)
    got = oracle.conflict_drive(wt, 1.0, -4.0, 0.0, 0.0, 0.0)
    OA, OB = wt[24:32].reshape(2, 4), wt[32:40].reshape(2, 4)
    want = 0.5 * (OA.sum(1) + OB.sum(1))
    for stim in range(9):
        np.testing.assert_allclose(got[stim], want, rtol=1e-15)


@pytest.mark.parametrize("wseed", [7, 8, 9, 10])
def test_correct_response_is_relevant_pathway_argmax(wseed):
    import torch
    wt = W.conflict_weights(wseed)
    got = oracle.conflict_correct(wt, 1.0, -4.0)
    WA, OA = torch.tensor(wt[:12]).view(4, 3), torch.tensor(wt[24:32]).view(2, 4)
    for stim in range(9):
        a = stim // 3
        resp = OA @ torch.sigmoid(WA[:, a] - 4.0)
        assert got[stim] == int(torch.argmax(resp).item())


def test_clone_identity_lca_equals_ddm_update():
    """With leak = competition = 0 (and no offset) each LCA unit's update is
    the DDM update with a = I*dt, b = sigma*sqrt(dt) -- bit for bit."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        x = rng.normal(0, 1, 2)
        inp = rng.normal(0, 2, 2)
        z = rng.normal(0, 1, 2)
        dt = rng.uniform(1e-3, 0.5)
        b = rng.uniform(0, 1) * math.sqrt(dt)
        out = oracle.lca_update(x, inp, 0.0, 0.0, dt, b, z)
        for i in range(2):
            assert out[i] == oracle.ddm_update(x[i], inp[i] * dt, b, z[i])


@pytest.mark.parametrize("leak,comp", [(0.5, 1.0), (1.0, 0.2), (0.3, 0.3)])
def test_linear_gaussian_moments(leak, comp):
    """With the threshold out of reach the linear LCA state after n steps is
    exactly Gaussian with the recursion's mean and covariance."""
    n, dt, noise = 12, 0.1, 0.4
    w = W.conflict(trials=9 * 8000, seed=21, leak=leak, comp=comp, noise=noise, thresh=1e300,
                   dt=dt, max_steps=n, n_bins=4, grid=np.array([[0.8, 1.3]]))
    out = oracle.run(w, dumps=True)
    xs = out["run_state"].reshape(-1, 9, 2)  # [trial/9, stim, unit]
    drive = oracle.conflict_drive(w["weights"], 1.0, -4.0, 0.0, 0.8, 1.3)
    b = noise * math.sqrt(dt)
    for stim in range(9):
        m, Cov = pins.lca_linear_moments(drive[stim], leak, comp, dt, b, n)
        sample = xs[:, stim, :]
        K = sample.shape[0]
        se = np.sqrt(np.diag(Cov) / K)
        assert np.all(np.abs(sample.mean(0) - m) < 4.5 * se), (stim, sample.mean(0), m)
        c = np.cov(sample.T)
        # sampling sd of a covariance entry is about sqrt((s_ii s_jj + s_ij^2) / K)
        sd = np.sqrt((np.outer(np.diag(Cov), np.diag(Cov)) + Cov ** 2) / K)
        assert np.all(np.abs(c - Cov) < 4.5 * sd), (stim, c, Cov)


def test_balanced_lca_difference_is_a_ddm():
    """leak = comp: x0 - x1 performs the DDM walk with drift I0 - I1 and
    noise sqrt(2) sigma (Bogacz et al. 2006); its distribution after n steps
    is N(n dt (I0 - I1), 2 n b^2)."""
    n, dt, noise = 15, 0.05, 0.3
    w = W.conflict(trials=9 * 6000, seed=5, leak=0.7, comp=0.7, noise=noise, thresh=1e300,
                   dt=dt, max_steps=n, n_bins=5, grid=np.array([[1.0, 1.0]]))
    xs = oracle.run(w, dumps=True)["run_state"].reshape(-1, 9, 2)
    drive = oracle.conflict_drive(w["weights"], 1.0, -4.0, 0.0, 1.0, 1.0)
    b = noise * math.sqrt(dt)
    for stim in range(9):
        d = xs[:, stim, 0] - xs[:, stim, 1]
        mean = n * dt * (drive[stim, 0] - drive[stim, 1])
        var = 2 * n * b * b
        assert abs(d.mean() - mean) < 4.5 * math.sqrt(var / d.size)
        assert abs(d.var() / var - 1) < 4.5 * math.sqrt(2 / d.size)


def test_noise_free_decision_matches_matrix_power():
    """sigma = 0: x_n = sum_{k<n} A^k dt I; the decision step is the first n
    where max(x_n) >= theta (matrix powers, not the update loop)."""
    leak, comp, dt, th = 0.5, 1.0, 0.1, 0.8
    w = W.conflict(trials=9, noise=0.0, grid=np.array([[0.6, 1.0]]))
    out = oracle.run(w, dumps=True)
    drive = oracle.conflict_drive(w["weights"], 1.0, -4.0, 0.0, 0.6, 1.0)
    A = np.eye(2) + dt * np.array([[-leak, -comp], [-comp, -leak]])
    for stim in range(9):
        acc = np.zeros(2)
        P = np.eye(2)
        for n in range(1, 1001):
            acc = acc + P @ (dt * drive[stim])
            P = A @ P
            if acc.max() >= th:
                break
        assert out["run_step"][stim] == n
        assert out["run_choice"][stim] == int(acc[1] > acc[0])
        np.testing.assert_allclose(out["run_state"][stim], acc, rtol=1e-12)


def test_nonneg_clipping_keeps_state_nonnegative():
    w = W.conflict(trials=900, seed=2, nonneg=1.0, noise=0.5, max_steps=200, n_bins=20)
    out = oracle.run(w, dumps=True)
    assert np.all(out["run_state"] >= 0.0)
    # the unclipped model goes negative somewhere on the same streams
    w0 = W.with_(w, params=w["params"].copy())
    w0["params"][W.LCA_P["nonneg"]] = 0.0
    assert np.any(oracle.run(w0, dumps=True)["run_state"] < 0.0)


def test_invariants_and_correct_counting():
    w = W.conflict(trials=900, seed=3)
    out = oracle.run(w, dumps=True)
    hist, st = out["hist"], out["stats"]
    T = w["trials"]
    assert np.all(hist.sum(axis=(1, 2)) + st[:, oracle.ST["undec"]] == T)
    corr = oracle.conflict_correct(w["weights"], 1.0, -4.0)
    ch = out["run_choice"].reshape(-1, T)
    stim = np.arange(T) % 9
    for s in range(ch.shape[0]):
        assert st[s, oracle.ST["correct"]] == (ch[s] == corr[stim]).sum()
    # decided runs end at or above threshold, in the direction of the choice
    xs = out["run_state"]
    dec = out["run_choice"] >= 0
    assert np.all(xs[dec].max(1) >= 0.8)
    assert np.all((xs[dec, 1] > xs[dec, 0]) == (out["run_choice"][dec] == 1))


def test_fp32_steps_close_to_fp64():
    w = W.conflict(trials=4000, seed=4, grid=W.control_grid(4))
    a = oracle.run(w)
    b = oracle.run(W.with_(w, precision=W.FP32_STEP))
    T = w["trials"]
    pa = a["hist"] / T
    pb = b["hist"] / T
    # paired streams: histogram L1 per setting well under 0.02
    assert np.abs(pa - pb).sum(axis=(1, 2)).max() < 0.02
