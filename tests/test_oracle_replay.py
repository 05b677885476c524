"""High-precision replay: a few runs recomputed at 50 significant digits
from the same Philox words.  This checks the oracle's FP64 rounding (state
within 1e-12 relative, same decision step unless flagged); the dynamics are
pinned by the distributional tests."""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W

mp.mp.dps = 50


def _normals(words):
    ma = ((int(words[1]) << 32) | int(words[0])) >> 11
    mb = ((int(words[3]) << 32) | int(words[2])) >> 11
    ua = mp.mpf(ma + 1) / mp.mpf(2) ** 53
    ub = mp.mpf(mb + 1) / mp.mpf(2) ** 53
    rho = mp.sqrt(-2 * mp.log(ua))
    phi = mp.mpf(6.283185307179586) * ub
    return rho * mp.cos(phi), rho * mp.sin(phi)


def _key(w):
    return [w["seed"] & 0xFFFFFFFF, w["seed"] >> 32]


@pytest.mark.parametrize("trial", range(6))
def test_ddm_replay(trial):
    w = W.ddm(trials=6, seed=17)
    traj, ch, fl = oracle.trajectory(w, 0, trial)
    a = mp.mpf(0.3 * 0.01)
    b = mp.mpf(1.0) * mp.sqrt(mp.mpf(0.01))
    x = mp.mpf(0)
    for n in range(1, traj.shape[0] + 1):
        z = _normals(oracle.philox([(n - 1) >> 1, trial, 0, 0], _key(w)))[(n - 1) & 1]
        x = x + a + b * z
        assert abs(float(x) - traj[n - 1, 0]) <= 1e-12 * max(1.0, abs(float(x)))
    if not fl:
        assert (x >= 1) if ch == 1 else (x <= -1)


@pytest.mark.parametrize("trial", range(9))
def test_lca_replay(trial):
    w = W.conflict(trials=9, seed=19, grid=np.array([[0.7, 1.0]]))
    traj, ch, fl = oracle.trajectory(w, 0, trial)
    drive = oracle.conflict_drive(w["weights"], 1.0, -4.0, 0.0, 0.7, 1.0)[trial % 9]
    I = [mp.mpf(drive[0]), mp.mpf(drive[1])]
    dt, leak, comp = mp.mpf(0.1), mp.mpf(0.5), mp.mpf(1.0)
    b = mp.mpf(0.1) * mp.sqrt(dt)
    x = [mp.mpf(0), mp.mpf(0)]
    for n in range(1, traj.shape[0] + 1):
        z = _normals(oracle.philox([n - 1, trial, 0, 0], _key(w)))
        x = [x[0] + (I[0] - leak * x[0] - comp * x[1]) * dt + b * z[0],
             x[1] + (I[1] - leak * x[1] - comp * x[0]) * dt + b * z[1]]
        for i in range(2):
            assert abs(float(x[i]) - traj[n - 1, i]) <= 1e-12 * max(1.0, abs(float(x[i])))
    if not fl and ch >= 0:
        assert max(x) >= mp.mpf(0.8) and (x[1] > x[0]) == (ch == 1)


@pytest.mark.parametrize("trial", range(2))
def test_rnn_replay(trial):
    """A coupled 64-unit rate network (W != 0), FP64, replayed at 50 digits
    from the same Philox words: p = W r with W row-major (unit i receives
    sum_j W[i][j] r_j), the Euler update of every unit, and the centred
    readout y <- y + dt R (r - 1/2) with the rates that fed the step.  Every
    unit and both readouts stay within 1e-11 of the oracle's FP64 trajectory
    (its rounding only), and the decision step and choice agree."""
    nu = 64
    wts = W.rnn_weights(nu, 7) * 2.0  # stronger coupling than N(0, 1/n)
    w = W.rnn(trials=2, seed=23, n_units=nu, weights=wts, max_steps=80, n_bins=10, thresh=0.25)
    traj, ch, fl = oracle.trajectory(w, 0, trial)
    Wm = [[mp.mpf(float(v)) for v in wts[i * nu:(i + 1) * nu]] for i in range(nu)]
    R = [[mp.mpf(float(v)) for v in wts[nu * nu + c * nu: nu * nu + (c + 1) * nu]] for c in (0, 1)]
    dt, noise, g = mp.mpf(0.05), mp.mpf(0.05), mp.mpf(1.0)
    b = noise * mp.sqrt(dt)
    u = []
    for m in range(nu // 2):
        u.extend(_normals(oracle.philox([m, trial, 0, 0x40000000], _key(w))))
    x = [mp.mpf(0)] * nu
    y = [mp.mpf(0), mp.mpf(0)]
    half = mp.mpf(1) / 2
    for n in range(1, traj.shape[0] + 1):
        xi = []
        for m in range(nu // 2):
            xi.extend(_normals(oracle.philox([n - 1, trial, 0, m], _key(w))))
        r = [1 / (1 + mp.exp(-v)) for v in x]
        p = [mp.fsum(Wm[i][j] * r[j] for j in range(nu)) for i in range(nu)]
        acc = [mp.fsum(R[c][j] * (r[j] - half) for j in range(nu)) for c in (0, 1)]
        x = [x[i] + dt * ((p[i] - x[i]) + g * u[i]) + b * xi[i] for i in range(nu)]
        y = [y[0] + dt * acc[0], y[1] + dt * acc[1]]
        row = traj[n - 1]
        assert abs(float(y[0]) - row[0]) <= 1e-11 and abs(float(y[1]) - row[1]) <= 1e-11, n
        assert max(abs(float(x[i]) - row[2 + i]) for i in range(nu)) <= 1e-11, n
    assert ch >= 0, "the run should decide within the cap"
    if not fl:
        assert max(y) >= mp.mpf(0.25) and (y[1] > y[0]) == (ch == 1)
        if traj.shape[0] > 1:
            prev = traj[-2]
            assert max(prev[0], prev[1]) < 0.25
